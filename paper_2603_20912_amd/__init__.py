"""MI355X (gfx950) particle-particle ladder term: Python front end of libppl.

The hot path (integral build from Cholesky vectors, the symmetric/antisymmetric
pair contraction, the packed Jacobi update) runs in the HIP library; this
package only marshals torch tensors into its C ABI (include/ppl.h).
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import (ppl_batch_plan, ppl_batch_query, ppl_batch_bind_workspace, ppl_batch_build,
                   ppl_batch_autotune, ppl_batch_contract, ppl_batch_graph_capture, ppl_batch_graph_capture_build,
                   ppl_batch_graph_launch, ppl_batch_destroy)
from ._lib import (ppl_mp2, ppl_mlp_create, ppl_mlp_workspace_bytes, ppl_mlp_bind_workspace,
                   ppl_mlp_param_count, ppl_mlp_init, ppl_mlp_set_params, ppl_mlp_get_params, ppl_mlp_grad,
                   ppl_mlp_train_step, ppl_mlp_sigma, ppl_mlp_samples, ppl_mlp_guess, ppl_mlp_destroy,
                   PPLError, ppl_bind_workspace, ppl_build_batch, ppl_contract, ppl_contract_tau, ppl_hhl,
                   ppl_ring, ppl_ring_scratch_bytes, ppl_ring_static,
                   ppl_destroy,
                   ppl_iter_opts_default, ppl_iterate, ppl_last_error, ppl_plan, ppl_plan_query,
                   ppl_profile_enable, ppl_profile_read, ppl_tile_count, ppl_tile_dims, ppl_version,
                   ppl_set_contract_config, ppl_autotune)

__all__ = ["PPL", "PPLError", "ppl_plan", "ppl_plan_query", "ppl_bind_workspace", "ppl_build_batch",
           "ppl_contract", "ppl_contract_tau", "ppl_hhl", "ppl_ring", "ppl_ring_scratch_bytes", "ppl_ring_static", "ring",
           "ppl_iterate", "ppl_destroy", "ppl_last_error", "ppl_tile_count", "ppl_tile_dims",
           "ppl_version", "ppl_iter_opts_default", "ppl_profile_enable", "ppl_profile_read",
           "ppl_set_contract_config", "ppl_autotune", "ppl_mp2", "MLP", "ppl_mlp_create",
           "ppl_mlp_workspace_bytes", "ppl_mlp_bind_workspace", "ppl_mlp_param_count", "ppl_mlp_init",
           "ppl_mlp_set_params", "ppl_mlp_get_params", "ppl_mlp_grad", "ppl_mlp_train_step",
           "ppl_mlp_sigma", "ppl_mlp_samples", "ppl_mlp_guess", "ppl_mlp_destroy", "Batch",
           "ppl_batch_plan", "ppl_batch_query", "ppl_batch_bind_workspace", "ppl_batch_build",
           "ppl_batch_autotune", "ppl_batch_contract", "ppl_batch_graph_capture", "ppl_batch_graph_capture_build",
           "ppl_batch_graph_launch", "ppl_batch_destroy"]


class PPL:
    """One planned problem with its device workspace (allocated by torch, owned here)."""

    def __init__(self, o, v, naux, prec="fp64", keep_fp64=False, hbm_budget=0, stream=None,
                 tile_contract=-1, device="cuda", build_scratch=0, diis_max=0, contract_only=False,
                 tune_cache=None, ring=False):
        if not torch.cuda.is_available():
            raise RuntimeError("PPL needs a HIP device (no CPU fallback)")
        self.o, self.v, self.naux = o, v, naux
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        if hbm_budget == 0:
            # the planner sizes the workspace from the device's free memory: hand the
            # blocks torch holds cached but unused back first, so that they count as free
            torch.cuda.empty_cache()
        self.plan = ppl_plan(o, v, naux, prec, keep_fp64, hbm_budget, self.stream, tile_contract, build_scratch,
                             diis_max, (_lib.PPL_PLAN_CONTRACT_ONLY if contract_only else 0)
                             | (_lib.PPL_PLAN_RING if ring else 0), tune_cache)
        self.info = ppl_plan_query(self.plan)
        nbytes = int(self.info["workspace_bytes"])
        self.workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        ppl_bind_workspace(self.plan, self.workspace)

    def build(self, L, batch=-1):
        ppl_build_batch(self.plan, L, batch)

    def contract(self, t2, R=None, alpha=1.0, beta=0.0, t1=None):
        """R = beta R + alpha PPL(t2), or PPL(t2 + t1 t1) when singles t1 [o][v] are given."""
        if R is None:
            R = torch.empty_like(t2)
        if t1 is None:
            ppl_contract(self.plan, t2, R, alpha, beta)
        else:
            ppl_contract_tau(self.plan, t2, t1, R, alpha, beta)
        return R

    def hhl(self, L, t2, R=None, alpha=1.0, beta=0.0):
        """R = beta R + alpha sum_kl (ki|lj) t_kl^ab."""
        if R is None:
            R = torch.empty_like(t2)
        ppl_hhl(self.plan, L, t2, R, alpha, beta)
        return R

    def iterate(self, L, e_occ, e_vir, t2, max_sweeps=100, tol=1e-7, start="mp2", switch_tol=0.0,
                stagnation=0.95, min_fp64_sweeps=2, diverge_factor=1e3, fail_on_noconv=True,
                history=True, raise_on_status=True, diis=0, hhl=False, ring=False):
        opts = ppl_iter_opts_default()
        opts.max_sweeps = int(max_sweeps)
        opts.tol = float(tol)
        opts.start = {"mp2": _lib.PPL_START_MP2, "given": _lib.PPL_START_GIVEN,
                      "checked": _lib.PPL_START_GIVEN_CHECKED}[start]
        opts.switch_tol = float(switch_tol)
        opts.stagnation = float(stagnation)
        opts.min_fp64_sweeps = int(min_fp64_sweeps)
        opts.diverge_factor = float(diverge_factor)
        opts.fail_on_noconv = int(bool(fail_on_noconv))
        opts.diis = int(diis)
        opts.hhl = int(bool(hhl))
        opts.ring = int(bool(ring))
        hist = (ctypes.c_double * max_sweeps)() if history else None
        if hist is not None:
            opts.history = ctypes.cast(hist, ctypes.POINTER(ctypes.c_double))
        rep = ppl_iterate(self.plan, L, e_occ, e_vir, t2, opts, raise_on_status=raise_on_status)
        n = rep["sweeps_lp"] + rep["sweeps_fp64"]
        rep["history"] = list(hist[:n]) if hist is not None else []
        return rep

    def contract_config(self):
        i = ppl_plan_query(self.plan)
        return (i["tile_contract"], i["splits_contract"], i["tile_contract_minus"], i["splits_contract_minus"])

    def set_contract_config(self, tile_plus, splits_plus, tile_minus, splits_minus):
        ppl_set_contract_config(self.plan, tile_plus, splits_plus, tile_minus, splits_minus)
        self.info = ppl_plan_query(self.plan)

    def autotune(self, reps=3):
        best = ppl_autotune(self.plan, reps)
        self.info = ppl_plan_query(self.plan)
        return best

    def profile(self, on=True):
        ppl_profile_enable(self.plan, on)

    def profile_read(self):
        return ppl_profile_read(self.plan)

    def mp2(self, L, e_occ, e_vir, t2_out=None):
        if t2_out is None:
            t2_out = torch.empty((self.o, self.o, self.v, self.v), dtype=torch.float64, device=L.device)
        e = ppl_mp2(self.plan, L, e_occ, e_vir, t2_out)
        return t2_out, e

    def close(self):
        if getattr(self, "plan", None) is not None:
            # the plan's enqueued work must end before its workspace goes back to torch
            self.stream.synchronize()
            ppl_destroy(self.plan)
            self.plan = None
        if getattr(self, "workspace", None) is not None:
            # hand the (large) workspace back to the device at once: left in torch's cache,
            # its segment could be split for a later small tensor and then never released
            self.workspace = None
            torch.cuda.empty_cache()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ring(L, t2, R=None, alpha=1.0, beta=0.0, stream=None, scratch=None):
    """R = beta R + alpha * (ring terms of the closed-shell doubles residual) on the GPU:
    Y_ij^ab + Y_ji^ba with Y_ij^ab = sum_kc [(2 t_ik^ac - t_ik^ca)(kc|jb) - t_ik^ac (kj|bc)
    - t_ik^cb (kj|ac)]. L is [naux][o+v][o+v], t2 and R [o][o][v][v], all FP64 on the
    device; the scratch (ppl_ring_scratch_bytes) is allocated here unless given."""
    o, v = t2.shape[0], t2.shape[2]
    naux = L.shape[0]
    if R is None:
        R = torch.empty_like(t2)
    if scratch is None:
        scratch = torch.empty(ppl_ring_scratch_bytes(o, v, naux), dtype=torch.uint8, device=t2.device)
    ppl_ring(o, v, naux, L, t2, R, scratch, alpha, beta, stream)
    return R


class MLP:
    """The learned-start network with its device workspace (parameters, Adam state, scratch)."""

    def __init__(self, max_batch=65536, seed=0, stream=None, device="cuda"):
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.h = ppl_mlp_create(128, max_batch, self.stream)
        self.max_batch = max_batch
        nbytes = ppl_mlp_workspace_bytes(self.h)
        self.workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        ppl_mlp_bind_workspace(self.h, self.workspace)
        ppl_mlp_init(self.h, seed)

    @property
    def n_params(self):
        return ppl_mlp_param_count(self.h)

    def get_params(self):
        return ppl_mlp_get_params(self.h)

    def set_params(self, flat):
        ppl_mlp_set_params(self.h, flat)

    def grad(self, X, Y):
        return ppl_mlp_grad(self.h, X, Y)

    def train_step(self, X, Y, lr=1e-3, want_loss=False):
        return ppl_mlp_train_step(self.h, X, Y, lr, want_loss=want_loss)

    def guess(self, eng, t_mp2, e_occ, e_vir, sigma=None, t2_out=None):
        if sigma is None:
            sigma = ppl_mlp_sigma(eng.plan, t_mp2)
        if t2_out is None:
            t2_out = torch.empty_like(t_mp2)
        ppl_mlp_guess(self.h, eng.plan, t_mp2, e_occ, e_vir, sigma, t2_out)
        return t2_out

    def close(self):
        if getattr(self, "h", None) is not None:
            self.stream.synchronize()
            ppl_mlp_destroy(self.h)
            self.h = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many uneven instances contracted by one persistent grouped launch (optionally a hipGraph)."""

    def __init__(self, shapes, prec="fp64", stream=None, device="cuda"):
        self.shapes = list(shapes)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.h = ppl_batch_plan(self.shapes, prec, self.stream)
        nbytes, _ = ppl_batch_query(self.h)
        self.workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        ppl_batch_bind_workspace(self.h, self.workspace)

    @property
    def n_items(self):
        return ppl_batch_query(self.h)[1]

    def build(self, Ls):
        self._L = list(Ls)          # the library keeps raw pointers
        ppl_batch_build(self.h, self._L)

    def autotune(self, reps=2):
        ppl_batch_autotune(self.h, reps)

    def contract(self, t2s, Rs):
        ppl_batch_contract(self.h, t2s, Rs)

    def capture(self, t2s, Rs, Ls=None):
        """Record the contraction (or, with Ls, the integral builds and the contraction) into a graph."""
        if Ls is None:
            self._graph_args = (list(t2s), list(Rs))
            ppl_batch_graph_capture(self.h, t2s, Rs)
        else:
            self._graph_args = (list(Ls), list(t2s), list(Rs))
            ppl_batch_graph_capture_build(self.h, Ls, t2s, Rs)

    def replay(self):
        ppl_batch_graph_launch(self.h)

    def close(self):
        if getattr(self, "h", None) is not None:
            self.stream.synchronize()
            ppl_batch_destroy(self.h)
            self.h = None
        if getattr(self, "workspace", None) is not None:
            self.workspace = None
            torch.cuda.empty_cache()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
