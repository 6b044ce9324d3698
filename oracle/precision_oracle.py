"""Emulation of the low-precision forms of the ladder term (test infrastructure).

TEST INFRASTRUCTURE. Only tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg may import or call this; the product never does.

Both forms evaluate the same sum as ppl_oracle.ppl (Sec. 2, eqs. (cholesky),
(vfunction-chol)) in the symmetric/antisymmetric pair form, but round the
operands where a low-precision GEMM pipeline has to:
  * "fp32":   operands rounded to FP32, products and sums exact (FP64 here);
  * "bf16x3": operands rounded to FP32, then x = hi + lo with hi = bf16(x),
              lo = bf16(x - hi) (round to nearest even), and x*y replaced by
              hi*hi + hi*lo + lo*hi (the lo*lo term dropped);
  * "bf16x6": operands rounded to FP32, then x = hi + mid + lo with hi = bf16(x),
              mid = bf16(x - hi), lo = bf16(x - hi - mid), and x*y replaced by the
              six products whose plane indices sum to at most two (hi*hi, hi*mid,
              mid*hi, mid*mid, hi*lo, lo*hi; mid*lo, lo*mid and lo*lo dropped).
These are the split-and-product schemes of Henry, Tang and Heinecke (ARITH 2019),
the low-precision products the paper's introduction points to (Sec. 1).
Rounding points: the virtual block of L (build operands), the integrals
G_ab[c][d] (FP32 accumulator output), V+- (operand precision), the packed
amplitudes S', A' (operand precision), and R (FP32 accumulator output).
Accumulation-order rounding inside the GEMMs is not emulated, so the GPU error
is expected at the emulated level up to a small factor.
"""
from __future__ import annotations

import numpy as np

__all__ = ["round_fp32", "round_bf16", "split_bf16x3", "split_bf16x6", "ppl_lowprec"]


def round_fp32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def round_bf16(x):
    """Round FP32 values to bfloat16 (nearest, ties to even) via their bit patterns."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def split_bf16x3(x):
    """x -> (hi, lo) with hi = bf16(fp32(x)), lo = bf16(fp32(x) - hi)."""
    x32 = round_fp32(x)
    hi = round_bf16(x32)
    lo = round_bf16(round_fp32(x32 - hi))
    return hi, lo


def split_bf16x6(x):
    """x -> (hi, mid, lo): hi = bf16(fp32(x)), mid = bf16(fp32(x) - hi), lo = bf16(fp32(x) - hi - mid)."""
    x32 = round_fp32(x)
    hi = round_bf16(x32)
    r1 = round_fp32(x32 - hi)
    mid = round_bf16(r1)
    lo = round_bf16(round_fp32(r1 - mid))
    return hi, mid, lo


def _mul_form(prec):
    if prec == "fp32":
        def prep(x):
            return (round_fp32(x),)

        def mm(a, b):                     # a @ b.T
            return a[0] @ b[0].T
    elif prec == "bf16x3":
        def prep(x):
            return split_bf16x3(x)

        def mm(a, b):
            return a[0] @ b[0].T + a[0] @ b[1].T + a[1] @ b[0].T
    elif prec == "bf16x6":
        def prep(x):
            return split_bf16x6(x)

        def mm(a, b):
            return (a[0] @ b[0].T + a[0] @ b[1].T + a[1] @ b[0].T
                    + a[1] @ b[1].T + a[0] @ b[2].T + a[2] @ b[0].T)
    else:
        raise ValueError(prec)
    return prep, mm


def ppl_lowprec(L, o, t, prec):
    """R_ij^ab of the pair method with the operand roundings of `prec` ("fp32" / "bf16x3" / "bf16x6")."""
    prep, mm = _mul_form(prec)
    L = np.asarray(L, dtype=np.float64)
    v = L.shape[1] - o
    oo = t.shape[0]
    Lvv = L[:, o:, o:]
    naux = L.shape[0]
    X = prep(Lvv.transpose(1, 2, 0).reshape(v * v, naux))         # rows (a,c), K = P
    # integrals of every pair a <= b, rounded to the FP32 accumulator
    au, bu = np.triu_indices(v)
    cu, du = np.triu_indices(v)
    cs, ds = np.triu_indices(v, 1)
    Vp = np.empty((au.size, cu.size))
    Vm = np.empty((au.size, cs.size))
    for a in range(v):
        rows = tuple(x[a * v:(a + 1) * v] for x in X)             # L_a[:, c]
        G = round_fp32(mm(rows, X).reshape(v, v, v))              # [c][b][d] = (ac|bd)
        for b in range(a, v):
            g = G[:, b, :]                                        # G_ab[c][d]
            p = a * v - a * (a + 1) // 2 + b
            Vp[p] = 0.5 * (g[cu, du] + g[du, cu])
            Vm[p] = 0.5 * (g[cs, ds] - g[ds, cs])
    keep_m = au < bu
    Vm = Vm[keep_m]
    # amplitudes in pair form
    iu, ju = np.triu_indices(oo)
    is_, js = np.triu_indices(oo, 1)
    w = np.where(cu == du, 1.0, 2.0)
    Sp = w * 0.5 * (t[iu, ju][:, cu, du] + t[iu, ju][:, du, cu])  # [N+][P+]
    Am = t[is_, js][:, cs, ds] - t[is_, js][:, ds, cs]             # [N-][P-]
    Rp = round_fp32(mm(prep(Sp), prep(Vp)))                        # [N+][P+]
    Rm = round_fp32(mm(prep(Am), prep(Vm))) if is_.size else np.zeros((0, cs.size))
    # unpack
    R = np.zeros_like(t)
    for q, (i, j) in enumerate(zip(iu, ju)):
        blk = np.zeros((v, v))
        blk[cu, du] = Rp[q]
        blk[du, cu] = Rp[q]
        if i != j:
            qm = np.nonzero((is_ == i) & (js == j))[0][0]
            anti = np.zeros((v, v))
            anti[cs, ds] = Rm[qm]
            anti[ds, cs] = -Rm[qm]
            R[i, j] = blk + anti
            R[j, i] = blk - anti
        else:
            R[i, i] = blk
    return R
