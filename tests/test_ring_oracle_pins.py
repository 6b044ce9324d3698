"""Pins of the closed-shell terms next to the ladder against the spin-orbital
linearized doubles equations. From closed-shell amplitudes t_ij^ab the spin-orbital
amplitudes are
    t_{I J}^{A B} = d(sI,sA) d(sJ,sB) t_ij^ab - d(sI,sB) d(sJ,sA) t_ij^ba
(s = spin, lower case = spatial index), and the antisymmetrized integrals are
<pq||rs> = (pr|qs) d(sp,sr) d(sq,ss) - (ps|qr) d(sp,ss) d(sq,sr). The textbook
spin-orbital terms
    ladder  1/2 sum_cd <ab||cd> t_ij^cd
    hole    1/2 sum_kl <kl||ij> t_kl^ab
    ring    P(ij) P(ab) sum_kc <kb||cj> t_ik^ac
must then have alpha-beta blocks equal to the closed-shell oracle functions ppl, hhl
and ring, and alpha-alpha blocks equal to R_ij^ab - R_ij^ba of the same functions.
This checks the spin adaptation of all three terms with no formula in common. The
closed-shell correlation energy sum V_ij^ab (2 t_ij^ab - t_ij^ba) is held the same way to
the spin-orbital energy 1/4 sum_IJAB <IJ||AB> t_IJ^AB."""
import numpy as np
import pytest

import oracle as O
import ppl_synth as S


def spin_orbital_terms(L, o, t):
    t_so, terms, _ = spin_orbital_parts(L, o, t)
    return t_so, terms


def spin_orbital_parts(L, o, t):
    n = L.shape[1]
    v = n - o
    eri = np.einsum("Ppq,Prs->pqrs", L, L)                       # (pq|rs)
    sp = np.repeat(np.arange(n), 2)                               # spatial index of spin orbital
    sg = np.tile([0, 1], n)                                       # spin of spin orbital
    same = (sg[:, None] == sg[None, :]).astype(float)
    # <pq|rs> = (pr|qs) d(sp,sr) d(sq,ss)
    g = eri[np.ix_(sp, sp, sp, sp)].transpose(0, 2, 1, 3) * same[:, None, :, None] * same[None, :, None, :]
    gA = g - g.transpose(0, 1, 3, 2)
    O2, V2 = slice(0, 2 * o), slice(2 * o, 2 * n)
    so, sv = sg[:2 * o], sg[2 * o:]
    io, iv = sp[:2 * o], sp[2 * o:] - o
    dIA = (so[:, None] == sv[None, :]).astype(float)              # d(sI, sA)
    tt = t[np.ix_(io, io, iv, iv)]                                # t_ij^ab over spin orbitals
    ts = t.transpose(0, 1, 3, 2)[np.ix_(io, io, iv, iv)]          # t_ij^ba
    t_so = dIA[:, None, :, None] * dIA[None, :, None, :] * tt - dIA[:, None, None, :] * dIA[None, :, :, None] * ts
    ladder = 0.5 * np.einsum("abcd,ijcd->ijab", gA[V2, V2, V2, V2], t_so)
    hole = 0.5 * np.einsum("klij,klab->ijab", gA[O2, O2, O2, O2], t_so)
    X = np.einsum("kbcj,ikac->ijab", gA[O2, V2, V2, O2], t_so)
    ring = X - X.transpose(1, 0, 2, 3) - X.transpose(0, 1, 3, 2) + X.transpose(1, 0, 3, 2)
    return t_so, {"ppl": ladder, "hhl": hole, "ring": ring}, gA[O2, O2, V2, V2]


def spin_orbital_energy(L, o, t):
    """1/4 sum_IJAB <IJ||AB> t_IJ^AB over the spin-orbital amplitudes of t."""
    t_so, _, g_oovv = spin_orbital_parts(L, o, t)
    return 0.25 * float(np.sum(g_oovv * t_so))


def blocks(R_so):
    ab = R_so[0::2, 1::2, 0::2, 1::2]        # i alpha, j beta, a alpha, b beta
    aa = R_so[0::2, 0::2, 0::2, 0::2]        # all alpha
    return ab, aa


@pytest.mark.parametrize("o,v,naux,seed", [(2, 3, 2, 0), (3, 4, 5, 1), (2, 5, 3, 2)])
def test_closed_shell_terms_are_the_spin_orbital_ones(o, v, naux, seed):
    s = S.make_system(o, v, naux, seed)
    t = S.make_amplitudes(o, v, seed + 10)
    t_so, terms = spin_orbital_terms(s["L"], o, t)
    # the spin-orbital amplitudes are antisymmetric (t is pair symmetric)
    assert np.allclose(t_so, -t_so.transpose(1, 0, 2, 3), atol=1e-14)
    assert np.allclose(t_so, -t_so.transpose(0, 1, 3, 2), atol=1e-14)
    for name, fn in (("ppl", O.ppl), ("hhl", O.hhl), ("ring", O.ring)):
        R = fn(s["L"], o, t)
        ab, aa = blocks(terms[name])
        scale = np.abs(R).max()
        assert np.abs(ab - R).max() < 1e-12 * scale, name
        assert np.abs(aa - (R - R.transpose(0, 1, 3, 2))).max() < 1e-12 * scale, name


def test_ring_is_pair_symmetric_and_linear():
    s = S.make_system(3, 6, 7, 3)
    t1 = S.make_amplitudes(3, 6, 4)
    t2 = S.make_amplitudes(3, 6, 5)
    R1, R2 = O.ring(s["L"], 3, t1), O.ring(s["L"], 3, t2)
    assert np.abs(R1 - R1.transpose(1, 0, 3, 2)).max() < 1e-14 * np.abs(R1).max()
    R12 = O.ring(s["L"], 3, 0.7 * t1 - 1.3 * t2)
    assert np.abs(R12 - (0.7 * R1 - 1.3 * R2)).max() < 1e-13 * np.abs(R12).max()
    # R(gamma L) = gamma^2 R(L): every integral is quadratic in L
    assert np.abs(O.ring(2.0 * s["L"], 3, t1) - 4.0 * R1).max() < 1e-13 * np.abs(R1).max()


def _ring_mutant(kind):
    def f(L, o, t):
        Lov, Loo, Lvv = L[:, :o, o:], L[:, :o, :o], L[:, o:, o:]
        J = np.einsum("Pkc,Pjb->kcjb", Lov, Lov)
        K = np.einsum("Pkj,Pbc->kjbc", Loo, Lvv)
        two = 1.0 if kind == "factor" else 2.0
        Y = np.einsum("ikac,kcjb->ijab", two * t - t.transpose(0, 1, 3, 2), J)
        Y -= np.einsum("ikac,kjbc->ijab", t, K)
        if kind != "dropped":
            Y -= np.einsum("ikcb,kjac->ijab", t, K) * (-1.0 if kind == "sign" else 1.0)
        if kind == "index":
            Y = (np.einsum("ikac,kcjb->ijab", 2.0 * t - t.transpose(0, 1, 3, 2), J.transpose(0, 3, 2, 1))
                 - np.einsum("ikac,kjbc->ijab", t, K) - np.einsum("ikcb,kjac->ijab", t, K))
        return Y + Y.transpose(1, 0, 3, 2)
    return f


@pytest.mark.parametrize("kind", ["factor", "dropped", "sign", "index"])
def test_planted_ring_mistakes_are_caught(kind):
    o, v = 2, 4
    s = S.make_system(o, v, 3, 6)
    t = S.make_amplitudes(o, v, 7)
    _, terms = spin_orbital_terms(s["L"], o, t)
    ab, _ = blocks(terms["ring"])
    assert np.abs(O.ring(s["L"], o, t) - ab).max() < 1e-12 * np.abs(ab).max()
    R = _ring_mutant(kind)(s["L"], o, t)
    assert np.abs(R - ab).max() > 1e-6 * np.abs(ab).max()


def test_ring_entry_matches_the_full_term():
    o, v = 3, 7
    s = S.make_system(o, v, 5, 8)
    t = S.make_amplitudes(o, v, 9)
    R = O.ring(s["L"], o, t)
    rng = np.random.default_rng(0)
    for _ in range(20):
        i, j = rng.integers(o, size=2)
        a, b = rng.integers(v, size=2)
        assert abs(O.ring_entry(s["L"], o, t, i, j, a, b) - R[i, j, a, b]) < 1e-13 * np.abs(R).max()


def test_terms_fixed_point_reduces_to_the_known_ones():
    # the tabulated operator reproduces the two dense solves that are written out directly
    s = S.make_system(2, 4, 6, 11, "contractive")
    a = O.fixed_point_terms(s["L"], 2, s["e_occ"], s["e_vir"], with_hhl=False, with_ring=False)
    assert np.abs(a - O.fixed_point(s["L"], 2, s["e_occ"], s["e_vir"])).max() < 1e-12 * np.abs(a).max()
    b = O.fixed_point_terms(s["L"], 2, s["e_occ"], s["e_vir"], with_hhl=True, with_ring=False)
    assert np.abs(b - O.fixed_point_hhl(s["L"], 2, s["e_occ"], s["e_vir"])).max() < 1e-12 * np.abs(b).max()


def test_iteration_with_ring_reaches_the_dense_fixed_point():
    # at this tiny size the plain iteration diverges with the ring terms (the contractive
    # generator keeps only the ladder's spectral radius below one); DIIS converges
    o, v, naux = 2, 5, 8
    s = S.make_system(o, v, naux, 12, "contractive")
    tstar = O.fixed_point_terms(s["L"], o, s["e_occ"], s["e_vir"])
    t, hist, _ = O.jacobi_diis(s["L"], o, s["e_occ"], s["e_vir"], m=6, max_sweeps=200, tol=1e-12,
                               with_hhl=True, with_ring=True)
    assert hist[-1] < 1e-12
    assert np.abs(t - tstar).max() < 1e-10 * np.abs(tstar).max()
    # the ring terms change the fixed point
    t0 = O.fixed_point_terms(s["L"], o, s["e_occ"], s["e_vir"], with_ring=False)
    assert np.abs(t0 - tstar).max() > 1e-4 * np.abs(tstar).max()


def test_plain_and_diis_iterations_with_ring_agree():
    o, v, naux = 6, 40, 120
    s = S.make_system(o, v, naux, 1, "contractive")
    tp, hp, Ep = O.jacobi(s["L"], o, s["e_occ"], s["e_vir"], max_sweeps=100, tol=1e-10, with_hhl=True,
                          with_ring=True)
    td, hd, Ed = O.jacobi_diis(s["L"], o, s["e_occ"], s["e_vir"], m=8, max_sweeps=100, tol=1e-10,
                               with_hhl=True, with_ring=True)
    assert hp[-1] < 1e-10 and hd[-1] < 1e-10 and len(hd) < len(hp)
    assert np.abs(tp - td).max() < 1e-8 * np.abs(tp).max()
    assert abs(Ep - Ed) < 1e-8


@pytest.mark.parametrize("o,v,naux,seed", [(2, 3, 2, 0), (3, 4, 5, 1), (2, 5, 3, 2), (3, 3, 4, 3)])
def test_energy_is_the_spin_orbital_one(o, v, naux, seed):
    # the closed-shell energy of random pair-symmetric amplitudes and of the MP2 ones
    s = S.make_system(o, v, naux, seed)
    V, D = O.mp2_parts(s["L"], o, s["e_occ"], s["e_vir"])
    for t in (S.make_amplitudes(o, v, seed + 20), V / D):
        e_so = spin_orbital_energy(s["L"], o, t)
        e = O.energy(V, t)
        assert abs(e - e_so) < 1e-12 * max(abs(e_so), np.abs(V).sum() * np.abs(t).max())
    # the MP2 energy of a closed shell is negative (every denominator is)
    assert O.energy(V, V / D) < 0.0


def _energy_mutant(kind):
    def f(V, t):
        tb = t.transpose(0, 1, 3, 2)
        if kind == "factor":                 # dropped factor 2 on the direct term
            return float(np.sum(V * (t - tb)))
        if kind == "swap":                   # t^ab written for t^ba in the exchange term
            return float(np.sum(V * (2.0 * t - t)))
        if kind == "sign":                   # exchange term added
            return float(np.sum(V * (2.0 * t + tb)))
        if kind == "half":                   # a spin-orbital prefactor carried over
            return 0.5 * float(np.sum(V * (2.0 * t - tb)))
        raise ValueError(kind)
    return f


@pytest.mark.parametrize("kind", ["factor", "swap", "sign", "half"])
def test_planted_energy_mistakes_are_caught(kind):
    o, v, naux = 3, 4, 5
    s = S.make_system(o, v, naux, 4)
    V, _ = O.mp2_parts(s["L"], o, s["e_occ"], s["e_vir"])
    t = S.make_amplitudes(o, v, 24)
    e_so = spin_orbital_energy(s["L"], o, t)
    assert abs(O.energy(V, t) - e_so) < 1e-12 * abs(e_so)
    assert abs(_energy_mutant(kind)(V, t) - e_so) > 1e-3 * abs(e_so)
