"""Seeded synthetic inputs for the particle-particle ladder (PPL) term.

This module only draws random numbers. It holds none of the method's arithmetic
(no integrals, no amplitudes, no contractions), so the CPU oracle and the HIP
path can both be fed from it without sharing any code of the method itself.

Recipe (Cholesky-decomposed ERI, eq. (cholesky); orbital order: the o occupied
orbitals first, then the v virtual ones):
  * L[P, p, q] = s_P * (A_P + A_P^T) / 2 with A_P ~ N(0, 1) over the n x n
    orbital space (n = o + v), so every Cholesky vector is symmetric in (p, q)
    as the real-orbital 8-fold ERI symmetry requires.
  * s_P = amp * exp(-P / (naux / 3)), P = 0 .. naux-1.
      - "literal":      amp = 0.3
      - "contractive":  amp = 6 / sqrt(v * naux)
    The literal amplitude makes the linearized doubles map diverge beyond the
    tiniest sizes (its spectral radius grows roughly like v * naux); the
    contractive amplitude scales the ladder operator by 400 / (v * naux) and
    keeps the spectral radius near 0.5-0.65 at every size, which is what runs
    that must converge use.
  * e_occ ~ U[-2.0, -0.5] (o values), e_vir ~ U[0.2, 5.0] (v values), each
    sorted ascending.
  * Draw order from numpy's PCG64 default_rng(seed): A (naux, n, n) as float64
    standard normals, then e_occ, then e_vir.
"""
from __future__ import annotations

import numpy as np

__all__ = ["make_system", "make_amplitudes", "batched_shapes", "training_shapes",
           "make_system_device", "make_amplitudes_device",
           "amplitude_scale", "MAX_ELEMS_GEN"]

# guard against accidentally asking for multi-100-GB host arrays
MAX_ELEMS_GEN = 2_000_000_000


def amplitude_scale(v: int, naux: int, variant: str) -> float:
    if variant == "literal":
        return 0.3
    if variant == "contractive":
        return 6.0 / np.sqrt(float(v) * float(naux))
    raise ValueError(f"unknown generator variant {variant!r}")


def make_system(o: int, v: int, naux: int, seed: int, variant: str = "literal",
                dtype=np.float64) -> dict:
    """Return {'L': [naux][n][n] float64, 'e_occ': [o], 'e_vir': [v], ...}."""
    if o < 1 or v < 1 or naux < 1:
        raise ValueError("o, v, naux must be >= 1")
    n = o + v
    if naux * n * n > MAX_ELEMS_GEN:
        raise ValueError("requested Cholesky tensor is too large to generate")
    rng = np.random.default_rng(seed)
    amp = amplitude_scale(v, naux, variant)
    L = np.empty((naux, n, n), dtype=np.float64)
    decay = naux / 3.0
    for P in range(naux):  # one vector at a time keeps the peak host memory at 1x
        A = rng.standard_normal((n, n))
        s = amp * np.exp(-P / decay)
        L[P] = (A + A.T) * (0.5 * s)
    e_occ = np.sort(rng.uniform(-2.0, -0.5, size=o))
    e_vir = np.sort(rng.uniform(0.2, 5.0, size=v))
    return {"o": o, "v": v, "naux": naux, "seed": seed, "variant": variant,
            "L": L.astype(dtype, copy=False), "e_occ": e_occ, "e_vir": e_vir}


def make_amplitudes(o: int, v: int, seed: int) -> np.ndarray:
    """A random pair-symmetric amplitude tensor t[i][j][a][b] = t[j][i][b][a].

    X ~ N(0,1) over (o, o, v, v); t = (X + X^pair) / 2 where X^pair swaps (i,a)
    with (j,b). This is only an input draw (the symmetry the amplitudes of a
    closed-shell doubles ansatz always carry, eq. (2)); no method arithmetic.
    """
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((o, o, v, v))
    return 0.5 * (X + X.transpose(1, 0, 3, 2))


def batched_shapes(n_inst: int = 32, seed: int = 4, o_range=(8, 24), v_range=(80, 240)):
    """Uneven instance list for the batched launch: o ~ U{o_range}, v ~ U{v_range},
    naux = 3v, instance k seeded 1000 + k (inclusive integer ranges)."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_inst):
        o = int(rng.integers(o_range[0], o_range[1] + 1))
        v = int(rng.integers(v_range[0], v_range[1] + 1))
        out.append({"o": o, "v": v, "naux": 3 * v, "seed": 1000 + k})
    return out


def training_shapes(n_inst: int = 200, seed: int = 5, o_range=(10, 30), v_range=(100, 300)):
    """Training-set instance list for the learned start: naux = 3v, seeds 2000 + k."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_inst):
        o = int(rng.integers(o_range[0], o_range[1] + 1))
        v = int(rng.integers(v_range[0], v_range[1] + 1))
        out.append({"o": o, "v": v, "naux": 3 * v, "seed": 2000 + k})
    return out


# ---------------------------------------------------------------- device-side draws
# The same recipe drawn directly in device memory with torch's device generator
# (Philox), for shapes whose host arrays would be tens of GB (the largest shape of
# the contraction benchmark, Tab. xc-split: L is 20 GB, t 39 GB). The numbers
# differ from the numpy draws of the same seed; only the distribution is shared.

def make_system_device(o: int, v: int, naux: int, seed: int, variant: str = "contractive",
                       device="cuda", chunk: int = 128) -> dict:
    """L [naux][n][n] float64 on `device` with the module's recipe (symmetrized standard
    normals scaled by amp * exp(-P / (naux / 3))), drawn `chunk` vectors at a time;
    e_occ, e_vir as in make_system."""
    import torch
    n = o + v
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    amp = amplitude_scale(v, naux, variant)
    L = torch.empty((naux, n, n), dtype=torch.float64, device=device)
    decay = naux / 3.0
    for p0 in range(0, naux, chunk):
        p1 = min(naux, p0 + chunk)
        A = torch.randn((p1 - p0, n, n), generator=g, dtype=torch.float64, device=device)
        s = amp * torch.exp(-torch.arange(p0, p1, dtype=torch.float64, device=device) / decay)
        L[p0:p1] = (A + A.transpose(1, 2)) * (0.5 * s)[:, None, None]
        del A
    e_occ = torch.sort(torch.rand(o, generator=g, dtype=torch.float64, device=device) * 1.5 - 2.0).values
    e_vir = torch.sort(torch.rand(v, generator=g, dtype=torch.float64, device=device) * 4.8 + 0.2).values
    return {"o": o, "v": v, "naux": naux, "seed": seed, "variant": variant, "L": L,
            "e_occ": e_occ, "e_vir": e_vir}


def make_amplitudes_device(o: int, v: int, seed: int, device="cuda"):
    """Pair-symmetric t[i][j][a][b] = (X + X^pair) / 2 with X ~ N(0, 1), drawn in place on
    `device`; the symmetrization runs one occupied row i at a time (temporary memory
    of (i+1) v^2 values)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    t = torch.empty((o, o, v, v), dtype=torch.float64, device=device)
    t.normal_(generator=g)
    for i in range(o):
        X = t[i, : i + 1]                          # t[i][j] for j <= i
        Y = t[: i + 1, i].transpose(1, 2)          # t[j][i]^T for j <= i
        S = (X + Y) * 0.5
        t[i, : i + 1] = S
        t[: i + 1, i] = S.transpose(1, 2)
        del X, Y, S
    return t
