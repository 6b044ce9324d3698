"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these tests re-types the oracle's own formula: each one checks it
against brute force, a closed form, a special case that reduces to a textbook
product, a symmetry of the integrals, linearity, an independent association of
the same sum, or an exact linear solve. The last block plants plausible
mistakes into copies of the oracle and shows that the pins catch them.
"""
import json
import os

import numpy as np
import pytest

import oracle as O
import ppl_synth as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def general_t(o, v, seed):
    """A t with no pair symmetry at all (the definition holds for any t)."""
    return np.random.default_rng(seed).standard_normal((o, o, v, v))


# ---------------------------------------------------------------- PPL itself
def test_hand_derived_golden():
    g = json.load(open(os.path.join(GOLDEN, "tiny_hand.json")))
    L = np.array(g["L"], dtype=float)
    for case in g["cases"]:
        R = O.ppl(L, g["o"], np.array(case["t"], dtype=float))
        np.testing.assert_array_equal(R, np.array(case["R"], dtype=float))


@pytest.mark.parametrize("o,v,naux,seed", [(2, 4, 3, 0), (3, 5, 2, 1), (1, 3, 4, 2)])
def test_ppl_matches_sixfold_loops(o, v, naux, seed):
    s = S.make_system(o, v, naux, seed)
    for t in (general_t(o, v, seed + 10), S.make_amplitudes(o, v, seed + 20)):
        R = O.ppl(s["L"], o, t)
        Rl = O.ppl_loops(s["L"], o, t)
        assert rel(R, Rl) < 1e-14


def test_naux1_is_a_sandwich_product():
    # one Cholesky vector M: R_ij = M t_ij M^T (two textbook matrix products)
    o, v = 3, 7
    s = S.make_system(o, v, 1, 3)
    M = s["L"][0, o:, o:]
    t = general_t(o, v, 4)
    R = O.ppl(s["L"], o, t)
    for i in range(o):
        for j in range(o):
            ref = np.linalg.multi_dot([M, t[i, j], M.T])
            assert rel(R[i, j], ref) < 1e-14


def test_identity_and_diagonal_cholesky_vectors():
    o, v, naux = 2, 6, 5
    rng = np.random.default_rng(7)
    n = o + v
    t = general_t(o, v, 8)
    # L^P restricted to the virtual block is the identity -> (ac|bd) = naux d_ac d_bd
    L = rng.standard_normal((naux, n, n))
    L = 0.5 * (L + L.transpose(0, 2, 1))
    L[:, o:, o:] = np.eye(v)
    assert rel(O.ppl(L, o, t), naux * t) < 1e-15
    # diagonal virtual block l^P -> R_ij^ab = (sum_P l^P_a l^P_b) t_ij^ab
    l = rng.standard_normal((naux, v))
    for P in range(naux):
        L[P, o:, o:] = np.diag(l[P])
    w = l.T @ l
    assert rel(O.ppl(L, o, t), w[None, None] * t) < 1e-14


def test_integral_symmetries():
    o, v, naux = 2, 6, 4
    s = S.make_system(o, v, naux, 11)
    Lvv = np.ascontiguousarray(s["L"][:, o:, o:])
    G = np.stack([O.eri_vvvv_for_a(Lvv, a) for a in range(v)])  # G[a][c][b][d] = (ac|bd)
    np.testing.assert_allclose(G, G.transpose(2, 3, 0, 1), rtol=0, atol=1e-15)  # (ac|bd) = (bd|ac)
    np.testing.assert_allclose(G, G.transpose(1, 0, 2, 3), rtol=0, atol=1e-15)  # (ac|bd) = (ca|bd)
    np.testing.assert_allclose(G, G.transpose(0, 1, 3, 2), rtol=0, atol=1e-15)  # (ac|bd) = (ac|db)


def test_pair_symmetry_of_result():
    o, v, naux = 4, 9, 12
    s = S.make_system(o, v, naux, 12)
    t = S.make_amplitudes(o, v, 13)
    R = O.ppl(s["L"], o, t)
    assert rel(R, R.transpose(1, 0, 3, 2)) < 1e-15


def test_linearity_in_t_and_homogeneity_in_L():
    o, v, naux = 3, 8, 10
    s = S.make_system(o, v, naux, 14)
    t1, t2 = general_t(o, v, 15), general_t(o, v, 16)
    al, be = 0.7, -1.9
    lhs = O.ppl(s["L"], o, al * t1 + be * t2)
    rhs = al * O.ppl(s["L"], o, t1) + be * O.ppl(s["L"], o, t2)
    assert rel(lhs, rhs) < 1e-14
    g = 1.7
    assert rel(O.ppl(g * s["L"], o, t1), g * g * O.ppl(s["L"], o, t1)) < 1e-14


@pytest.mark.parametrize("o,v,naux", [(10, 100, 300)])
def test_independent_association_realistic(o, v, naux):
    s = S.make_system(o, v, naux, 1)
    V, D = O.mp2_parts(s["L"], o, s["e_occ"], s["e_vir"])
    t = V / D
    assert rel(O.ppl(s["L"], o, t), O.ppl_factored(s["L"], o, t)) < 1e-13


def test_sampled_entries_match_full():
    o, v, naux = 5, 20, 60
    s = S.make_system(o, v, naux, 0)
    t = S.make_amplitudes(o, v, 1)
    R = O.ppl(s["L"], o, t)
    rng = np.random.default_rng(2)
    idx = [tuple(int(x) for x in (rng.integers(o), rng.integers(o), rng.integers(v), rng.integers(v)))
           for _ in range(50)]
    got = O.ppl_sampled(s["L"], o, t, idx)
    ref = np.array([R[k] for k in idx])
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-13 * np.abs(R).max())


# ---------------------------------------------------------------- MP2, energy
def test_mp2_parts_against_loops():
    o, v, naux = 3, 4, 5
    s = S.make_system(o, v, naux, 21)
    L = s["L"]
    V, D = O.mp2_parts(L, o, s["e_occ"], s["e_vir"])
    for i in range(o):
        for j in range(o):
            for a in range(v):
                for b in range(v):
                    ref = sum(L[P, i, o + a] * L[P, j, o + b] for P in range(naux))
                    assert abs(V[i, j, a, b] - ref) < 1e-14
                    dref = s["e_occ"][i] + s["e_occ"][j] - s["e_vir"][a] - s["e_vir"][b]
                    assert D[i, j, a, b] == dref
    assert (D < 0).all()      # occupied below virtual: every denominator is negative
    assert rel(V, V.transpose(1, 0, 3, 2)) == 0.0


def test_energy_against_loops_and_mp2_closed_form():
    o, v, naux = 3, 4, 6
    s = S.make_system(o, v, naux, 22)
    V, D = O.mp2_parts(s["L"], o, s["e_occ"], s["e_vir"])
    t = V / D
    e_loop = 0.0
    for i in range(o):
        for j in range(o):
            for a in range(v):
                for b in range(v):
                    e_loop += V[i, j, a, b] * (2 * t[i, j, a, b] - t[i, j, b, a])
    assert abs(O.energy(V, t) - e_loop) < 1e-13 * abs(e_loop)
    # closed-shell MP2 energy is negative for negative denominators
    assert O.energy(V, t) < 0.0


# ---------------------------------------------------------------- iteration
def test_jacobi_reaches_the_exact_fixed_point():
    o, v, naux = 5, 20, 60
    s = S.make_system(o, v, naux, 0, "contractive")
    args = (s["L"], o, s["e_occ"], s["e_vir"])
    t, hist, E = O.jacobi(*args, max_sweeps=200, tol=1e-11)
    assert hist[-1] < 1e-11
    tstar = O.fixed_point(*args)
    # the fixed point satisfies its own equation
    V, D = O.mp2_parts(*args)
    assert rel(D * tstar - O.ppl(s["L"], o, tstar), V) < 1e-13
    assert rel(t, tstar) < 1e-9
    assert abs(E - O.energy(V, tstar)) < 1e-9


def test_diis_with_one_vector_is_the_plain_iteration():
    o, v, naux = 3, 12, 36
    s = S.make_system(o, v, naux, 7, "contractive")
    args = (s["L"], o, s["e_occ"], s["e_vir"])
    t1, h1, E1 = O.jacobi(*args, max_sweeps=15, tol=0.0)
    t2, h2, E2 = O.jacobi_diis(*args, m=1, max_sweeps=15, tol=0.0)
    assert h1 == h2 and np.array_equal(t1, t2) and E1 == E2


def test_diis_terminates_on_the_affine_map():
    # The Jacobi map is affine; with the whole history DIIS minimizes the residual over a
    # growing Krylov space (it is GMRES on (I - M) t = D^-1 V), so it reaches the exact
    # fixed point once the space is exhausted: o = 1, v = 3 leaves 6 pair-symmetric
    # unknowns, hence at most 6 extrapolations after the first sweep (8 sweeps in all).
    o, v, naux = 1, 3, 4
    s = S.make_system(o, v, naux, 7, "contractive")
    args = (s["L"], o, s["e_occ"], s["e_vir"])
    tstar = O.fixed_point(*args)
    t, hist, _ = O.jacobi_diis(*args, m=8, max_sweeps=30, tol=1e-13)
    assert len(hist) <= 8 and hist[-1] < 1e-13
    assert rel(t, tstar) < 1e-13
    # the plain iteration (spectral radius near 0.97) is still far away after as many sweeps
    _, hj, _ = O.jacobi(*args, max_sweeps=len(hist), tol=0.0)
    assert hj[-1] > 1e-5


def test_diis_reaches_the_same_fixed_point_in_fewer_sweeps():
    o, v, naux = 4, 24, 72
    s = S.make_system(o, v, naux, 7, "contractive")
    args = (s["L"], o, s["e_occ"], s["e_vir"])
    tstar = O.fixed_point(*args)
    tj, hj, _ = O.jacobi(*args, max_sweeps=200, tol=1e-10)
    td, hd, Ed = O.jacobi_diis(*args, m=8, max_sweeps=200, tol=1e-10)
    assert hd[-1] < 1e-10 and rel(td, tstar) < 1e-9 and rel(tj, tstar) < 1e-9
    assert 2 * len(hd) < len(hj)
    V, _ = O.mp2_parts(*args)
    assert abs(Ed - O.energy(V, tstar)) < 1e-9


def test_diis_converges_where_jacobi_diverges():
    o, v, naux = 3, 16, 48
    s = S.make_system(o, v, naux, 2, "literal")
    args = (s["L"], o, s["e_occ"], s["e_vir"])
    assert O.spectral_radius(*args, iters=150) > 1.3
    _, hj, _ = O.jacobi(*args, max_sweeps=30, tol=0.0)
    assert hj[-1] > 10 * hj[0]
    t, hd, _ = O.jacobi_diis(*args, m=8, max_sweeps=60, tol=1e-10)
    assert hd[-1] < 1e-10 and rel(t, O.fixed_point(*args)) < 1e-9


def test_generator_variants_rho():
    o, v, naux = 5, 20, 60
    lit = S.make_system(o, v, naux, 0, "literal")
    con = S.make_system(o, v, naux, 0, "contractive")
    rl = O.spectral_radius(lit["L"], o, lit["e_occ"], lit["e_vir"], iters=300)
    rc = O.spectral_radius(con["L"], o, con["e_occ"], con["e_vir"], iters=300)
    assert rl > 1.2                   # the literal amplitude diverges already here
    assert 0.3 < rc < 0.7             # the contractive amplitude converges
    # K scales with amp^2 while D is unchanged
    kappa2 = (S.amplitude_scale(v, naux, "contractive") / 0.3) ** 2
    assert abs(rc - kappa2 * rl) < 1e-6 * rl
    _, hist, _ = O.jacobi(lit["L"], o, lit["e_occ"], lit["e_vir"], max_sweeps=12, tol=0.0)
    assert hist[-1] > 10 * hist[0]


def test_nominal_flops_counts_pairs():
    for o, v, naux in [(3, 5, 7), (4, 6, 2)]:
        Pp = sum(1 for a in range(v) for b in range(v) if a <= b)
        Pm = sum(1 for a in range(v) for b in range(v) if a < b)
        Np = sum(1 for i in range(o) for j in range(o) if i <= j)
        Nm = sum(1 for i in range(o) for j in range(o) if i < j)
        f = O.nominal_flops(o, v, naux)
        assert f["build"] == 2 * naux * v * v * Pp
        assert f["contract"] == 2 * (Pp * Pp * Np + Pm * Pm * Nm)
        assert f["dense"] == 2 * (naux + o * o) * v ** 4


# ---------------------------------------------------------------- planted mistakes
def _ppl_wrong_eri_pairing(L, o, t):          # <ab|cd> read as (ab|cd)
    Lvv = L[:, o:, o:]
    return np.einsum("Pab,Pcd,ijcd->ijab", Lvv, Lvv, t)


def _ppl_transposed_t(L, o, t):               # t_ij^dc instead of t_ij^cd
    return O.ppl(L, o, t.transpose(0, 1, 3, 2))


def _ppl_dropped_vector(L, o, t):             # last Cholesky vector dropped
    return O.ppl(L[:-1], o, t)


def _ppl_wrong_block(L, o, t):                # occupied offset forgotten
    Lvv = L[:, :L.shape[1] - o, :L.shape[1] - o]
    return np.einsum("Pac,Pbd,ijcd->ijab", Lvv, Lvv, t)


@pytest.mark.parametrize("mutant", [_ppl_wrong_eri_pairing, _ppl_transposed_t,
                                    _ppl_dropped_vector, _ppl_wrong_block])
def test_planted_mistakes_are_caught(mutant):
    o, v, naux = 2, 4, 3
    s = S.make_system(o, v, naux, 0)
    t = general_t(o, v, 10)
    assert rel(mutant(s["L"], o, t), O.ppl_loops(s["L"], o, t)) > 1e-3


def _diis_variant(L, o, e_occ, e_vir, mistake, m=8, max_sweeps=30, tol=1e-13):
    """The DIIS iteration with one planted mistake, to show that the DIIS pins catch it."""
    V, D = O.mp2_parts(L, o, e_occ, e_vir)
    t = V / D
    Ts, Es, hist = [], [], []
    for _ in range(max_sweeps):
        t_new = (V + O.ppl(L, o, t)) / D
        e = t_new - t
        hist.append(float(np.linalg.norm(e)))
        if hist[-1] < tol:
            return t_new, hist
        Ts.append(t if mistake == "extrapolate_inputs" else t_new)
        Es.append(t_new if mistake == "errors_are_iterates" else e)
        Ts, Es = Ts[-m:], Es[-m:]
        n = len(Es)
        A = np.zeros((n + 1, n + 1))
        A[:n, :n] = [[float(np.sum(x * y)) for y in Es] for x in Es]
        A[:n, n] = A[n, :n] = -1.0
        rhs = np.zeros(n + 1)
        rhs[n] = 1.0 if mistake == "constraint_sign" else -1.0
        c = np.linalg.lstsq(A, rhs, rcond=None)[0][:n]
        t = sum(ci * Ti for ci, Ti in zip(c, Ts))
    return t, hist


@pytest.mark.parametrize("mistake", ["extrapolate_inputs", "errors_are_iterates", "constraint_sign"])
def test_planted_diis_mistakes_are_caught(mistake):
    o, v, naux = 1, 3, 4
    s = S.make_system(o, v, naux, 7, "contractive")
    args = (s["L"], o, s["e_occ"], s["e_vir"])
    t, hist = _diis_variant(*args, mistake)
    # the affine-termination pin: exact fixed point within 8 sweeps
    assert not (len(hist) <= 8 and hist[-1] < 1e-13 and rel(t, O.fixed_point(*args)) < 1e-13)


# ---------------------------------------------------------------- CCSD terms next to the ladder
def test_hhl_matches_loops():
    o, v, naux = 3, 2, 2
    s = S.make_system(o, v, naux, 5)
    L = s["L"]
    t = general_t(o, v, 6)
    R = np.zeros((o, o, v, v))
    for i in range(o):
        for j in range(o):
            for a in range(v):
                for b in range(v):
                    for k in range(o):
                        for l in range(o):
                            for P in range(naux):
                                R[i, j, a, b] += L[P, k, i] * L[P, l, j] * t[k, l, a, b]
    assert rel(O.hhl(L, o, t), R) < 1e-14


def test_hhl_special_cases():
    # one Cholesky vector: R_ab = Loo^T T_ab Loo for every virtual pair (a, b)
    o, v = 4, 3
    s = S.make_system(o, v, 1, 8)
    t = general_t(o, v, 9)
    Loo = s["L"][0, :o, :o]
    ref = np.einsum("ki,klab,lj->ijab", Loo, t, Loo)
    assert rel(O.hhl(s["L"], o, t), ref) < 1e-14
    # one occupied orbital: R_00^ab = (00|00) t_00^ab
    s1 = S.make_system(1, 5, 6, 10)
    t1 = general_t(1, 5, 11)
    assert rel(O.hhl(s1["L"], 1, t1), np.sum(s1["L"][:, 0, 0] ** 2) * t1) < 1e-14
    # only the occupied block of L enters
    s2 = S.make_system(3, 5, 4, 12)
    L2 = s2["L"].copy()
    L2[:, 3:, :] *= -7.0
    L2[:, :, 3:] += 1.0
    t2 = general_t(3, 5, 13)
    assert np.array_equal(O.hhl(s2["L"], 3, t2), O.hhl(L2, 3, t2))


def test_hhl_keeps_pair_symmetry():
    o, v, naux = 4, 5, 6
    s = S.make_system(o, v, naux, 14)
    t = S.make_amplitudes(o, v, 15)
    R = O.hhl(s["L"], o, t)
    assert rel(R, R.transpose(1, 0, 3, 2)) < 1e-14


def test_ppl_tau_against_independent_association():
    o, v, naux = 3, 6, 5
    s = S.make_system(o, v, naux, 16)
    t2 = S.make_amplitudes(o, v, 17)
    t1 = np.random.default_rng(18).standard_normal((o, v))
    # singles switched off: the plain ladder
    assert np.array_equal(O.ppl_tau(s["L"], o, t2, np.zeros((o, v))), O.ppl(s["L"], o, t2))
    # the singles part: sum_cd (ac|bd) t_i^c t_j^d = sum_P (L^P t1^T)_ai (L^P t1^T)_bj
    Lvv = s["L"][:, o:, o:]
    Y = Lvv @ t1.T                                   # [P][a][i]
    quad = np.einsum("Pai,Pbj->ijab", Y, Y)
    assert rel(O.ppl_tau(s["L"], o, t2, t1) - O.ppl(s["L"], o, t2), quad) < 1e-13
    # tau keeps the pair symmetry of t2
    tt = O.tau(t2, t1)
    assert np.array_equal(tt, tt.transpose(1, 0, 3, 2))


def _hhl_swapped_integral(L, o, t):
    Loo = L[:, :o, :o]
    W = np.einsum("Pkl,Pij->klij", Loo, Loo)          # (kl|ij) instead of (ki|lj)
    return np.einsum("klij,klab->ijab", W, t)


def _hhl_transposed_amplitudes(L, o, t):
    return O.hhl(L, o, t.transpose(1, 0, 2, 3))


@pytest.mark.parametrize("mutant", [_hhl_swapped_integral, _hhl_transposed_amplitudes])
def test_planted_hhl_mistakes_are_caught(mutant):
    o, v, naux = 3, 2, 2
    s = S.make_system(o, v, naux, 5)
    t = general_t(o, v, 6)
    assert rel(mutant(s["L"], o, t), O.hhl(s["L"], o, t)) > 1e-3


def test_iteration_with_hhl_reaches_the_dense_fixed_point():
    o, v, naux = 4, 12, 36
    s = S.make_system(o, v, naux, 5, "contractive")
    args = (s["L"], o, s["e_occ"], s["e_vir"])
    tstar = O.fixed_point_hhl(*args)
    V, D = O.mp2_parts(*args)
    # the dense operator (built from einsum definitions) and the two term functions agree
    assert rel(D * tstar - O.ppl(s["L"], o, tstar) - O.hhl(s["L"], o, tstar), V) < 1e-13
    t, hist, E = O.jacobi(*args, max_sweeps=200, tol=1e-11, with_hhl=True)
    assert hist[-1] < 1e-11 and rel(t, tstar) < 1e-9
    # the hole-hole ladder moves the fixed point by far more than the tolerance
    assert rel(O.fixed_point(*args), tstar) > 1e-2
    # DIIS reaches it too, where the plain sweeps crawl
    s3 = S.make_system(3, 16, 48, 6, "contractive")
    a3 = (s3["L"], 3, s3["e_occ"], s3["e_vir"])
    _, hj, _ = O.jacobi(*a3, max_sweeps=40, tol=1e-11, with_hhl=True)
    td, hd, _ = O.jacobi_diis(*a3, m=8, max_sweeps=60, tol=1e-11, with_hhl=True)
    assert hj[-1] > 1e-6 and hd[-1] < 1e-11 and rel(td, O.fixed_point_hhl(*a3)) < 1e-9
