"""Learned start of the amplitude iteration: data, training and evaluation driver.

Every arithmetic step runs in libppl: converged amplitudes come from
ppl_iterate (FP64), first-order amplitudes from ppl_mp2, features and targets
from ppl_mlp_samples, training from ppl_mlp_train_step (FP32 forward/backward
kernels + Adam), the guess from ppl_mlp_guess (BF16 MFMA inference). This
module only chooses instances, sample indices and minibatch order.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import PPL, MLP, ppl_mlp_samples, ppl_mlp_sigma


def upload_system(sysd, device="cuda"):
    return {k: torch.from_numpy(np.ascontiguousarray(sysd[k])).to(device) for k in ("L", "e_occ", "e_vir")}


def converge(sysd, tol=1e-9, max_sweeps=300, device="cuda"):
    """FP64 Jacobi from MP2 to `tol`; returns device tensors and the report."""
    o, v, naux = sysd["o"], sysd["v"], sysd["naux"]
    d = upload_system(sysd, device)
    eng = PPL(o, v, naux, prec="fp64")
    t_mp2, e_mp2 = eng.mp2(d["L"], d["e_occ"], d["e_vir"])
    t_star = torch.empty_like(t_mp2)
    rep = eng.iterate(d["L"], d["e_occ"], d["e_vir"], t_star, max_sweeps=max_sweeps, tol=tol)
    sigma = ppl_mlp_sigma(eng.plan, t_mp2)
    return {"eng": eng, "d": d, "t_mp2": t_mp2, "t_star": t_star, "sigma": sigma, "report": rep,
            "e_mp2": e_mp2, "o": o, "v": v}


def sample(inst, n_samples, gen: torch.Generator, device="cuda"):
    """Features and targets at n_samples random elements of the instance."""
    o, v = inst["o"], inst["v"]
    total = o * o * v * v
    n = min(n_samples, total)
    idx = torch.randperm(total, generator=gen)[:n].to(device=device, dtype=torch.int64)
    X = torch.empty((n, 4), dtype=torch.float32, device=device)
    Y = torch.empty((n,), dtype=torch.float32, device=device)
    ppl_mlp_samples(inst["eng"].plan, inst["t_mp2"], inst["t_star"], inst["d"]["e_occ"], inst["d"]["e_vir"],
                    inst["sigma"], idx, X, Y)
    return X, Y


def train(mlp: MLP, X, Y, steps=2000, batch=4096, lr=1e-3, seed=0, log_every=0):
    """Adam on random minibatches of the pooled samples; returns the loss history (every log step)."""
    gen = torch.Generator().manual_seed(seed)
    n = Y.numel()
    hist = []
    for it in range(steps):
        sel = torch.randint(0, n, (min(batch, n),), generator=gen).to(X.device)
        xb = X.index_select(0, sel).contiguous()
        yb = Y.index_select(0, sel).contiguous()
        want = bool(log_every) and (it % log_every == 0 or it == steps - 1)
        loss = mlp.train_step(xb, yb, lr=lr, want_loss=want)
        if want:
            hist.append((it, loss))
    return hist


def time_to_tol(sysd, start, mlp=None, tol=1e-7, prec="fp64", keep_fp64=False, max_sweeps=300,
                device="cuda", switch_tol=1e-5):
    """Wall time and sweeps from inputs in HBM to a converged residual below tol.

    start: 'mp2' (plain), 'learned' (network guess, unchecked) or 'checked'
    (network guess, restarted from MP2 when its first residual is larger).
    The timed region covers the first-order amplitudes, the network guess, the
    integral builds and every sweep.
    """
    o, v, naux = sysd["o"], sysd["v"], sysd["naux"]
    d = upload_system(sysd, device)
    eng = PPL(o, v, naux, prec=prec, keep_fp64=keep_fp64)
    t = torch.empty((o, o, v, v), dtype=torch.float64, device=device)
    tm = torch.empty_like(t) if start != "mp2" else None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if start == "mp2":
        rep = eng.iterate(d["L"], d["e_occ"], d["e_vir"], t, max_sweeps=max_sweeps, tol=tol, start="mp2",
                          switch_tol=switch_tol, raise_on_status=False)
    else:
        eng.mp2(d["L"], d["e_occ"], d["e_vir"], tm)
        mlp.guess(eng, tm, d["e_occ"], d["e_vir"], t2_out=t)
        rep = eng.iterate(d["L"], d["e_occ"], d["e_vir"], t, max_sweeps=max_sweeps, tol=tol,
                          start="checked" if start == "checked" else "given", switch_tol=switch_tol,
                          raise_on_status=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rep = dict(rep)
    rep["seconds"] = dt
    rep["sweeps"] = rep["sweeps_lp"] + rep["sweeps_fp64"]
    eng.close()
    return rep, t
