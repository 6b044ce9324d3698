"""Plain FP64 CPU oracle of the particle-particle ladder (PPL) hot path.

TEST INFRASTRUCTURE. Only tests/, __graft_entry__.smoke() and the cpu_baseline
leg of bench.py may import or call anything in this package. The product
(paper_2603_20912_amd and its HIP library) never imports it and shares no code
with it: every quantity here is written straight from its definition in the
paper (Sec. 2, eqs. (ppl-term), (cholesky), (vfunction-chol)) in NumPy float64,
with no packing, blocking over summation indices or precision tricks.

Conventions (readings of the paper, all stated in the design doc as well):
  * L[P, p, q], P = 0..naux-1, over all n = o + v orbitals, occupied first.
  * Chemist's notation: the physicist's <ab|cd> of eq. (ppl-term) is (ac|bd),
    and eq. (cholesky) builds it as (ac|bd) = sum_P L^P_ac L^P_bd.
  * Amplitudes and results are t[i][j][a][b] = t_ij^ab (C-contiguous).
  * The ladder term enters the spin-free closed-shell vector function with
    coefficient +1 (eq. (vfunction-chol)):
        R_ij^ab = sum_{c,d} (ac|bd) t_ij^cd.
  * V_ij^ab = (ia|jb) from the occupied-virtual block of the same L,
    D_ij^ab = e_i + e_j - e_a - e_b, MP2 start t = V / D.
  * Linearized doubles (Jacobi) iteration t <- (V + PPL(t)) / D, residual
    r = ||t_new - t||_F over the full o*o*v*v tensor (absolute, FP64).
  * Correlation energy E = sum_{ijab} V_ij^ab (2 t_ij^ab - t_ij^ba).

Parity pins of every function live in tests/test_oracle_pins.py and, for the terms and
the energy checked against the spin-orbital equations, tests/test_ring_oracle_pins.py.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "vv_block", "ov_block", "eri_vvvv_for_a", "ppl", "ppl_loops", "ppl_factored",
    "ppl_sampled", "ppl_entry", "oo_block", "tau", "ppl_tau", "hhl", "ring", "ring_entry", "mp2_parts", "mp2_amplitudes", "energy", "jacobi_sweep",
    "jacobi", "jacobi_diis", "fixed_point", "fixed_point_hhl", "fixed_point_terms", "spectral_radius", "nominal_flops",
]


# ---------------------------------------------------------------------------
# integrals (eq. (cholesky))
# ---------------------------------------------------------------------------
def vv_block(L: np.ndarray, o: int) -> np.ndarray:
    """Virtual-virtual block L[P, o+a, o+c] of the Cholesky vectors."""
    return L[:, o:, o:]


def ov_block(L: np.ndarray, o: int) -> np.ndarray:
    """Occupied-virtual block L[P, i, o+a] of the Cholesky vectors."""
    return L[:, :o, o:]


def eri_vvvv_for_a(Lvv: np.ndarray, a: int) -> np.ndarray:
    """W[c, b, d] = (ac|bd) = sum_P L^P_ac L^P_bd for one fixed virtual a (eq. (cholesky)).

    Lvv is the C-contiguous virtual block [P][a][c].
    """
    naux, v, _ = Lvv.shape
    W = Lvv[:, a, :].T @ Lvv.reshape(naux, v * v)        # [c][(b,d)]
    return W.reshape(v, v, v)


# ---------------------------------------------------------------------------
# the ladder term (eqs. (ppl-term), (vfunction-chol))
# ---------------------------------------------------------------------------
def ppl(L: np.ndarray, o: int, t: np.ndarray) -> np.ndarray:
    """R_ij^ab = sum_cd (ac|bd) t_ij^cd, evaluated one virtual a at a time.

    For each a the integrals (ac|bd) are first summed over P (eq. (cholesky)),
    then contracted over (c, d) with the amplitudes (eq. (vfunction-chol)).
    The loop over a only bounds host memory; it touches no summation.
    """
    L = np.asarray(L, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    v = L.shape[1] - o
    oo = t.shape[0]
    assert t.shape == (oo, oo, v, v)
    Lvv = np.ascontiguousarray(vv_block(L, o))
    R = np.empty_like(t)
    for a in range(v):
        W = eri_vvvv_for_a(Lvv, a)                       # [c][b][d]
        R[:, :, a, :] = np.tensordot(t, W, axes=([2, 3], [0, 2]))  # sum over c, d -> [i][j][b]
    return R


def ppl_loops(L: np.ndarray, o: int, t: np.ndarray) -> np.ndarray:
    """The same sum written as explicit loops over i, j, a, b, c, d and P (tiny sizes only)."""
    naux, n, _ = L.shape
    v = n - o
    oo = t.shape[0]
    R = np.zeros((oo, oo, v, v))
    for i in range(oo):
        for j in range(oo):
            for a in range(v):
                for b in range(v):
                    s = 0.0
                    for c in range(v):
                        for d in range(v):
                            eri = 0.0
                            for P in range(naux):
                                eri += L[P, o + a, o + c] * L[P, o + b, o + d]
                            s += eri * t[i, j, c, d]
                    R[i, j, a, b] = s
    return R


def ppl_factored(L: np.ndarray, o: int, t: np.ndarray) -> np.ndarray:
    """Independent association of the same sum: R_ij = sum_P L^P t_ij (L^P)^T.

    This is the O(x o^2 v^3) order of Sec. 2 (no v^4 intermediate). It shares no
    intermediate with ppl() and so cross-checks it at realistic sizes.
    """
    Lvv = vv_block(np.asarray(L, dtype=np.float64), o)
    oo = t.shape[0]
    v = Lvv.shape[1]
    R = np.zeros_like(t, dtype=np.float64)
    T = t.reshape(oo * oo, v, v)
    Rr = R.reshape(oo * oo, v, v)
    for P in range(Lvv.shape[0]):
        M = Lvv[P]
        Rr += np.matmul(np.matmul(M, T), M.T)   # [a][c] t[c][d] [d][b]
    return R


def ppl_entry(La: np.ndarray, Lb: np.ndarray, tij: np.ndarray) -> float:
    """One R_ij^ab from the slices it depends on: La[P, c] = L^P_ac and Lb[P, d] = L^P_bd
    (virtual c, d), tij[c, d] = t_ij^cd. G[c, d] = (ac|bd) = sum_P L^P_ac L^P_bd, then
    R = sum_cd G[c, d] t_ij^cd. Lets full-size results be checked from O(naux v) data."""
    G = np.asarray(La, dtype=np.float64).T @ np.asarray(Lb, dtype=np.float64)   # [c][d]
    return float(np.sum(G * np.asarray(tij, dtype=np.float64)))


def ppl_sampled(L: np.ndarray, o: int, t: np.ndarray, idx) -> np.ndarray:
    """R_ij^ab at a list of (i, j, a, b) samples, each from its own (ac|bd) slab.

    Cost per sample is O(naux v^2), so full-size results can be spot-checked.
    """
    Lvv = vv_block(np.asarray(L, dtype=np.float64), o)
    out = np.empty(len(idx))
    for k, (i, j, a, b) in enumerate(idx):
        out[k] = ppl_entry(Lvv[:, a, :], Lvv[:, b, :], t[i, j])
    return out


# ---------------------------------------------------------------------------
# terms of the CCSD residual next to the ladder (not part of the paper's hot
# path; standard closed-shell CCSD, written from the definitions)
# ---------------------------------------------------------------------------
def oo_block(L: np.ndarray, o: int) -> np.ndarray:
    """Occupied-occupied block L[P, k, i] of the Cholesky vectors."""
    return L[:, :o, :o]


def tau(t2: np.ndarray, t1: np.ndarray) -> np.ndarray:
    """tau_ij^ab = t_ij^ab + t_i^a t_j^b, the amplitudes that carry the singles into the
    particle-particle ladder of CCSD (t1 is [i][a])."""
    t1 = np.asarray(t1, dtype=np.float64)
    return np.asarray(t2, dtype=np.float64) + t1[:, None, :, None] * t1[None, :, None, :]


def ppl_tau(L: np.ndarray, o: int, t2: np.ndarray, t1: np.ndarray) -> np.ndarray:
    """The ladder term of CCSD: R_ij^ab = sum_cd (ac|bd) tau_ij^cd."""
    return ppl(L, o, tau(t2, t1))


def hhl(L: np.ndarray, o: int, t: np.ndarray) -> np.ndarray:
    """Hole-hole ladder R_ij^ab = sum_kl (ki|lj) t_kl^ab with (ki|lj) = sum_P L^P_ki L^P_lj."""
    Loo = np.asarray(oo_block(np.asarray(L, dtype=np.float64), o))
    naux = Loo.shape[0]
    X = Loo.reshape(naux, o * o)                       # [P][(k,i)]
    W = (X.T @ X).reshape(o, o, o, o)                  # W[k, i, l, j] = (ki|lj)
    t = np.asarray(t, dtype=np.float64)
    v = t.shape[2]
    M = W.transpose(1, 3, 0, 2).reshape(o * o, o * o)  # [(i,j)][(k,l)]
    return (M @ t.reshape(o * o, v * v)).reshape(o, o, v, v)


def ring(L: np.ndarray, o: int, t: np.ndarray) -> np.ndarray:
    """Ring (particle-hole) terms of the closed-shell linearized doubles residual,
    R_ij^ab = Y_ij^ab + Y_ji^ba with
        Y_ij^ab = sum_kc [ (2 t_ik^ac - t_ik^ca) (kc|jb) - t_ik^ac (kj|bc) - t_ik^cb (kj|ac) ],
    the closed-shell (alpha-beta) block of the spin-orbital term
    P(ij) P(ab) sum_kc <kb||cj> t_ik^ac (checked against that definition in the pins)."""
    L = np.asarray(L, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    Lov = L[:, :o, o:]
    Loo = L[:, :o, :o]
    Lvv = L[:, o:, o:]
    J = np.einsum("Pkc,Pjb->kcjb", Lov, Lov)          # (kc|jb)
    K = np.einsum("Pkj,Pbc->kjbc", Loo, Lvv)          # (kj|bc)
    Y = (np.einsum("ikac,kcjb->ijab", 2.0 * t - t.transpose(0, 1, 3, 2), J)
         - np.einsum("ikac,kjbc->ijab", t, K)
         - np.einsum("ikcb,kjac->ijab", t, K))
    return Y + Y.transpose(1, 0, 3, 2)


def ring_entry(L: np.ndarray, o: int, t: np.ndarray, i: int, j: int, a: int, b: int) -> float:
    """One element R_ij^ab of ring(), from the slices of L it needs (for large sizes)."""
    L = np.asarray(L, dtype=np.float64)
    Lov, Loo, Lvv = L[:, :o, o:], L[:, :o, :o], L[:, o:, o:]

    def Y(i, j, a, b):
        Jb = np.einsum("Pkc,P->kc", Lov, Lov[:, j, b])          # (kc|jb) over k, c
        Kb = np.einsum("Pk,Pc->kc", Loo[:, :, j], Lvv[:, b, :])  # (kj|bc)
        Ka = np.einsum("Pk,Pc->kc", Loo[:, :, j], Lvv[:, a, :])  # (kj|ac)
        tia = t[i, :, a, :]                                      # t_ik^ac over k, c
        tic = t[i, :, :, a]                                      # t_ik^ca
        tib = t[i, :, :, b]                                      # t_ik^cb
        return float(np.sum((2.0 * tia - tic) * Jb) - np.sum(tia * Kb) - np.sum(tib * Ka))

    return Y(i, j, a, b) + Y(j, i, b, a)


# ---------------------------------------------------------------------------
# MP2 start, denominators, energy
# ---------------------------------------------------------------------------
def mp2_parts(L: np.ndarray, o: int, e_occ: np.ndarray, e_vir: np.ndarray):
    """V_ij^ab = (ia|jb) = sum_P L^P_ia L^P_jb and D_ij^ab = e_i + e_j - e_a - e_b."""
    Lov = ov_block(np.asarray(L, dtype=np.float64), o)      # [P][i][a]
    naux, oo, v = Lov.shape
    X = Lov.transpose(1, 2, 0).reshape(oo * v, naux)        # [(i,a)][P]
    V = (X @ X.T).reshape(oo, v, oo, v).transpose(0, 2, 1, 3).copy()  # [i][j][a][b]
    e_occ = np.asarray(e_occ, dtype=np.float64)
    e_vir = np.asarray(e_vir, dtype=np.float64)
    D = (e_occ[:, None, None, None] + e_occ[None, :, None, None]
         - e_vir[None, None, :, None] - e_vir[None, None, None, :])
    return V, D


def mp2_amplitudes(L, o, e_occ, e_vir) -> np.ndarray:
    """First-order amplitudes t = V / D."""
    V, D = mp2_parts(L, o, e_occ, e_vir)
    return V / D


def energy(V: np.ndarray, t: np.ndarray) -> float:
    """E = sum_{ijab} V_ij^ab (2 t_ij^ab - t_ij^ba), the closed-shell form of the spin-orbital
    doubles energy 1/4 sum <IJ||AB> t_IJ^AB (pinned to it in tests/test_ring_oracle_pins.py)."""
    return float(np.sum(V * (2.0 * t - t.transpose(0, 1, 3, 2))))


# ---------------------------------------------------------------------------
# linearized doubles iteration (the PPL-only vector function with the Fock
# denominators), its exact fixed point and its contraction rate
# ---------------------------------------------------------------------------
def jacobi_sweep(L, o, V, D, t, with_hhl: bool = False, with_ring: bool = False):
    """One simultaneous update t_new = (V + PPL(t) [+ HHL(t)] [+ RING(t)]) / D; returns
    (t_new, ||t_new - t||_F)."""
    g = V + ppl(L, o, t)
    if with_hhl:
        g = g + hhl(L, o, t)
    if with_ring:
        g = g + ring(L, o, t)
    t_new = g / D
    return t_new, float(np.linalg.norm(t_new - t))


def jacobi(L, o, e_occ, e_vir, t0=None, max_sweeps: int = 100, tol: float = 1e-7, with_hhl: bool = False,
           with_ring: bool = False):
    """Iterate from t0 (MP2 when None) until r < tol or max_sweeps; with_hhl adds the
    hole-hole ladder and with_ring the ring terms to every sweep.

    Returns (t, residual_history, E(t)).
    """
    V, D = mp2_parts(L, o, e_occ, e_vir)
    t = V / D if t0 is None else np.array(t0, dtype=np.float64)
    hist = []
    for _ in range(max_sweeps):
        t, r = jacobi_sweep(L, o, V, D, t, with_hhl, with_ring)
        hist.append(r)
        if not np.isfinite(r) or r < tol:
            break
    return t, hist, energy(V, t)


def jacobi_diis(L, o, e_occ, e_vir, t0=None, m: int = 6, max_sweeps: int = 100, tol: float = 1e-7,
                with_hhl: bool = False, with_ring: bool = False):
    """Jacobi iteration accelerated by direct inversion in the iterative subspace
    (DIIS; P. Pulay, Chem. Phys. Lett. 73, 393 (1980)).

    Sweep k maps its input t_k to t'_k = (V + PPL(t_k)) / D with error e_k = t'_k - t_k;
    r_k = ||e_k||_F is the same residual the plain iteration reports. Unless r_k < tol,
    the next input is t_{k+1} = sum_i c_i t'_i over the last m sweeps, where c minimizes
    ||sum_i c_i e_i||_F subject to sum_i c_i = 1, i.e. solves
        [ B   -1 ] [c     ]   [ 0 ]
        [ -1^T 0 ] [lambda] = [-1 ],   B_ij = <e_i, e_j>_F.
    A singular system drops the oldest sweep and is solved again. With m = 1 this is
    the plain iteration. Returns (t, residual_history, E(t)), t = t'_k of the last sweep.

    Singular is read numerically: the system, with B divided by its largest diagonal
    entry, has an LU pivot (partial pivoting) below 1e-14.
    """
    import scipy.linalg
    V, D = mp2_parts(L, o, e_occ, e_vir)
    t = V / D if t0 is None else np.array(t0, dtype=np.float64)
    Ts, Es, hist = [], [], []
    for _ in range(max_sweeps):
        t_new, _ = jacobi_sweep(L, o, V, D, t, with_hhl, with_ring)
        e = t_new - t
        r = float(np.linalg.norm(e))
        hist.append(r)
        if not np.isfinite(r) or r < tol:
            t = t_new
            break
        Ts.append(t_new)
        Es.append(e)
        if len(Ts) > m:
            Ts.pop(0)
            Es.pop(0)
        while True:
            n = len(Es)
            A = np.zeros((n + 1, n + 1))
            for i in range(n):
                for j in range(n):
                    A[i, j] = float(np.sum(Es[i] * Es[j]))
            A[:n, :n] /= max(abs(A[i, i]) for i in range(n))
            A[:n, n] = -1.0
            A[n, :n] = -1.0
            rhs = np.zeros(n + 1)
            rhs[n] = -1.0
            lu, piv = scipy.linalg.lu_factor(A, check_finite=False)
            if np.min(np.abs(np.diag(lu))) >= 1e-14:
                c = scipy.linalg.lu_solve((lu, piv), rhs)[:n]
                break
            if n == 1:                 # a zero error vector: the sweep's own amplitudes
                c = np.ones(1)
                break
            Ts.pop(0)
            Es.pop(0)
        t = sum(ci * Ti for ci, Ti in zip(c, Ts))
    return t, hist, energy(V, t)


def fixed_point_hhl(L, o, e_occ, e_vir) -> np.ndarray:
    """Exact solution of t = (V + PPL(t) + HHL(t)) / D by one dense solve over all
    (i, j, a, b): the operator is K[(ijab),(klcd)] = (ac|bd) d_ik d_jl + (ki|lj) d_ac d_bd.
    Tiny sizes only ((o v)^2 x (o v)^2 system)."""
    L = np.asarray(L, dtype=np.float64)
    Lvv, Loo = vv_block(L, o), oo_block(L, o)
    v = Lvv.shape[1]
    Kv = np.einsum("Pac,Pbd->abcd", Lvv, Lvv)          # (ac|bd)
    Ko = np.einsum("Pki,Plj->ijkl", Loo, Loo)          # (ki|lj)
    Io, Iv = np.eye(o), np.eye(v)
    K = (np.einsum("abcd,ik,jl->ijabklcd", Kv, Io, Io) + np.einsum("ijkl,ac,bd->ijabklcd", Ko, Iv, Iv))
    n = o * o * v * v
    V, D = mp2_parts(L, o, e_occ, e_vir)
    A = np.diag(D.ravel()) - K.reshape(n, n)
    return np.linalg.solve(A, V.ravel()).reshape(o, o, v, v)


def fixed_point_terms(L, o, e_occ, e_vir, with_hhl: bool = True, with_ring: bool = True) -> np.ndarray:
    """Exact solution of t = (V + PPL(t) [+ HHL(t)] [+ RING(t)]) / D by one dense solve:
    the linear operator is tabulated column by column, applying the term functions to
    every unit tensor. Tiny sizes only ((o v)^2 x (o v)^2 system)."""
    L = np.asarray(L, dtype=np.float64)
    V, D = mp2_parts(L, o, e_occ, e_vir)
    shape = V.shape
    n = V.size
    M = np.empty((n, n))
    for q in range(n):
        e = np.zeros(n)
        e[q] = 1.0
        e = e.reshape(shape)
        g = ppl(L, o, e)
        if with_hhl:
            g = g + hhl(L, o, e)
        if with_ring:
            g = g + ring(L, o, e)
        M[:, q] = g.ravel()
    A = np.diag(D.ravel()) - M
    return np.linalg.solve(A, V.ravel()).reshape(shape)


def fixed_point(L, o, e_occ, e_vir) -> np.ndarray:
    """Exact solution of t = (V + PPL(t)) / D by one dense linear solve per (i, j).

    With K[(a,b),(c,d)] = (ac|bd), the fixed point obeys (diag(D_ij) - K) t_ij = V_ij.
    Tiny sizes only (v^2 x v^2 systems).
    """
    Lvv = vv_block(np.asarray(L, dtype=np.float64), o)
    v = Lvv.shape[1]
    K = np.einsum("Pac,Pbd->abcd", Lvv, Lvv).reshape(v * v, v * v)
    V, D = mp2_parts(L, o, e_occ, e_vir)
    oo = V.shape[0]
    t = np.empty_like(V)
    for i in range(oo):
        for j in range(oo):
            A = np.diag(D[i, j].ravel()) - K
            t[i, j] = np.linalg.solve(A, V[i, j].ravel()).reshape(v, v)
    return t


def spectral_radius(L, o, e_occ, e_vir, iters: int = 200, seed: int = 0) -> float:
    """Power-iteration estimate of rho of the Jacobi map x -> PPL(x) / D on pair-symmetric x."""
    V, D = mp2_parts(L, o, e_occ, e_vir)
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(V.shape)
    x = 0.5 * (x + x.transpose(1, 0, 3, 2))
    x /= np.linalg.norm(x)
    lam = 0.0
    for _ in range(iters):
        y = ppl(L, o, x) / D
        lam = float(np.linalg.norm(y))
        if lam == 0.0:
            return 0.0
        x = y / lam
    return lam


# ---------------------------------------------------------------------------
# flop accounting of the symmetric/antisymmetric pair method (reference counts)
# ---------------------------------------------------------------------------
def nominal_flops(o: int, v: int, naux: int) -> dict:
    """Useful flops of one PPL evaluation in the i<=j / a<=b pair method.

    build    = 2 naux v^2 P+     (G_ab = L_a^T L_b for every a <= b)
    contract = 2 (P+^2 N+ + P-^2 N-)
    with P+- = v(v+-1)/2, N+- = o(o+-1)/2; dense = 2 (naux + o^2) v^4.
    """
    Pp, Pm = v * (v + 1) // 2, v * (v - 1) // 2
    Np, Nm = o * (o + 1) // 2, o * (o - 1) // 2
    build = 2.0 * naux * v * v * Pp
    contract = 2.0 * (Pp * Pp * Np + Pm * Pm * Nm)
    dense = 2.0 * (naux + o * o) * float(v) ** 4
    return {"build": build, "contract": contract, "eval": build + contract, "dense": dense}
