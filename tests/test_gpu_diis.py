"""GPU tests of the DIIS-accelerated iteration (ppl_iterate with opts.diis = m)
against the oracle's jacobi_diis and the exact fixed point: the same residual
history sweep by sweep, finite termination on a tiny affine map, convergence
where the plain iteration diverges, and the mixed-precision run reaching the
FP64 fixed point in fewer sweeps."""
import sys

import numpy as np
import pytest

import oracle as O
import ppl_synth as S

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2603_20912_amd as P
    return P


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def run(P, s, m, prec="fp64", keep=False, diis_max=8, **kw):
    o, v, naux = s["o"], s["v"], s["naux"]
    eng = P.PPL(o, v, naux, prec=prec, keep_fp64=keep, diis_max=diis_max)
    t = torch.zeros((o, o, v, v), dtype=torch.float64, device="cuda")
    rep = eng.iterate(dev(s["L"]), dev(s["e_occ"]), dev(s["e_vir"]), t, diis=m, **kw)
    eng.close()
    return rep, t.cpu().numpy()


def test_diis_history_matches_oracle(P):
    o, v, naux = 4, 24, 72
    say(f"iterate fp64 diis 8 to 1e-10 ({o},{v},{naux}) contractive seed 7")
    s = S.make_system(o, v, naux, 7, "contractive")
    rep, t = run(P, s, 8, max_sweeps=200, tol=1e-10)
    tref, href, Eref = O.jacobi_diis(s["L"], o, s["e_occ"], s["e_vir"], m=8, max_sweeps=200, tol=1e-10)
    say(f"  sweeps {len(rep['history'])} (oracle {len(href)}), dropped {rep['diis_dropped']}")
    assert rep["status"] == 0 and len(rep["history"]) == len(href)
    h, hr = np.array(rep["history"]), np.array(href)
    # residuals agree to rounding until they approach it
    big = hr > 1e-8
    assert np.all(np.abs(h[big] - hr[big]) <= 1e-6 * hr[big])
    assert rel(t, tref) < 1e-9
    assert rel(t, O.fixed_point(s["L"], o, s["e_occ"], s["e_vir"])) < 1e-8
    assert abs(rep["energy"] - Eref) < 1e-9


def test_diis_with_one_vector_is_the_plain_iteration(P):
    o, v, naux = 3, 12, 36
    say(f"iterate fp64 diis 1 vs plain ({o},{v},{naux})")
    s = S.make_system(o, v, naux, 7, "contractive")
    r1, t1 = run(P, s, 1, max_sweeps=15, tol=0.0)
    r0, t0 = run(P, s, 0, max_sweeps=15, tol=0.0, diis_max=0)
    assert r1["history"] == r0["history"] and np.array_equal(t1, t0)


def test_diis_terminates_on_the_affine_map(P):
    say("iterate fp64 diis 8 (1,3,4): exact fixed point within 8 sweeps")
    s = S.make_system(1, 3, 4, 7, "contractive")
    rep, t = run(P, s, 8, max_sweeps=30, tol=1e-13)
    assert rep["status"] == 0 and len(rep["history"]) <= 8
    assert rel(t, O.fixed_point(s["L"], 1, s["e_occ"], s["e_vir"])) < 1e-12


def test_diis_converges_where_jacobi_diverges(P):
    o, v, naux = 3, 16, 48
    say(f"iterate fp64 diis 8 ({o},{v},{naux}) literal seed 2 (plain iteration diverges)")
    s = S.make_system(o, v, naux, 2, "literal")
    r0, _ = run(P, s, 0, max_sweeps=60, tol=1e-10, diverge_factor=1e3, raise_on_status=False)
    assert r0["status"] == -6
    rep, t = run(P, s, 8, max_sweeps=60, tol=1e-10)
    say(f"  diis: {len(rep['history'])} sweeps, residual {rep['residual']:.2e}")
    assert rep["status"] == 0
    assert rel(t, O.fixed_point(s["L"], o, s["e_occ"], s["e_vir"])) < 1e-9


@pytest.mark.parametrize("prec", ["bf16x3", "fp32", "bf16x6"])
def test_mixed_diis_reaches_fp64_fixed_point_in_fewer_sweeps(P, prec):
    o, v, naux = 10, 100, 300
    say(f"mixed {prec} -> fp64 with diis 8 to 1e-7 ({o},{v},{naux}) contractive")
    s = S.make_system(o, v, naux, 1, "contractive")
    rd, td = run(P, s, 8, prec=prec, keep=True, max_sweeps=200, tol=1e-7)
    rp, _ = run(P, s, 0, prec=prec, keep=True, diis_max=0, max_sweeps=200, tol=1e-7)
    nd = rd["sweeps_lp"] + rd["sweeps_fp64"]
    npl = rp["sweeps_lp"] + rp["sweeps_fp64"]
    say(f"  diis: lp {rd['sweeps_lp']} fp64 {rd['sweeps_fp64']}; plain: lp {rp['sweeps_lp']} fp64 {rp['sweeps_fp64']}")
    assert rd["status"] == 0 and rd["residual"] < 1e-7 and rd["sweeps_fp64"] >= 2
    assert 3 * nd <= 2 * npl
    tstar, _, Estar = O.jacobi(s["L"], o, s["e_occ"], s["e_vir"], max_sweeps=200, tol=1e-11)
    assert rel(td, tstar) < 1e-6
    assert abs(rd["energy"] - Estar) < 1e-6


def test_diis_beyond_the_plan_capacity_is_rejected(P):
    s = S.make_system(2, 8, 24, 1, "contractive")
    with pytest.raises(P.PPLError) as e:
        run(P, s, 5, diis_max=4, max_sweeps=5, tol=0.0)
    assert e.value.code == -1


def test_iteration_with_hhl_matches_oracle(P):
    o, v, naux = 4, 12, 36
    say(f"iterate fp64 with the hole-hole ladder to 1e-11 ({o},{v},{naux}) contractive seed 5")
    s = S.make_system(o, v, naux, 5, "contractive")
    rep, t = run(P, s, 0, diis_max=0, max_sweeps=200, tol=1e-11, hhl=True)
    tref, href, Eref = O.jacobi(s["L"], o, s["e_occ"], s["e_vir"], max_sweeps=200, tol=1e-11, with_hhl=True)
    assert rep["status"] == 0 and len(rep["history"]) == len(href)
    h, hr = np.array(rep["history"]), np.array(href)
    # residuals agree to rounding (an absolute 1e-16 of amplitudes of order one) until they approach it
    assert np.all(np.abs(h - hr) <= 1e-9 * hr + 1e-14)
    assert rel(t, O.fixed_point_hhl(s["L"], o, s["e_occ"], s["e_vir"])) < 1e-9
    assert abs(rep["energy"] - Eref) < 1e-10


def test_diis_with_hhl_matches_oracle(P):
    o, v, naux = 3, 16, 48
    say(f"iterate fp64 diis 8 with the hole-hole ladder ({o},{v},{naux}) contractive seed 6")
    s = S.make_system(o, v, naux, 6, "contractive")
    rep, t = run(P, s, 8, max_sweeps=60, tol=1e-11, hhl=True)
    tref, href, _ = O.jacobi_diis(s["L"], o, s["e_occ"], s["e_vir"], m=8, max_sweeps=60, tol=1e-11, with_hhl=True)
    assert rep["status"] == 0 and len(rep["history"]) == len(href)
    assert rel(t, O.fixed_point_hhl(s["L"], o, s["e_occ"], s["e_vir"])) < 1e-9


@pytest.mark.parametrize("prec", ["bf16x3", "fp32", "bf16x6"])
def test_mixed_iteration_with_hhl(P, prec):
    o, v, naux = 10, 100, 300
    say(f"mixed {prec} -> fp64 with the hole-hole ladder and diis 8 to 1e-7 ({o},{v},{naux})")
    s = S.make_system(o, v, naux, 1, "contractive")
    rep, t = run(P, s, 8, prec=prec, keep=True, max_sweeps=200, tol=1e-7, hhl=True)
    assert rep["status"] == 0 and rep["residual"] < 1e-7 and rep["sweeps_fp64"] >= 2
    tstar, _, Estar = O.jacobi(s["L"], o, s["e_occ"], s["e_vir"], max_sweeps=200, tol=1e-10, with_hhl=True)
    assert rel(t, tstar) < 1e-6
    assert abs(rep["energy"] - Estar) < 1e-6


def test_hhl_iteration_needs_a_resident_plan(P):
    o, v, naux = 4, 30, 20
    s = S.make_system(o, v, naux, 7, "contractive")
    eng = P.PPL(o, v, naux)
    budget = eng.info["workspace_bytes"] // 3
    eng.close()
    eng = P.PPL(o, v, naux, hbm_budget=budget)
    assert eng.info["resident"] == 0
    t = torch.zeros((o, o, v, v), dtype=torch.float64, device="cuda")
    with pytest.raises(P.PPLError) as e:
        eng.iterate(dev(s["L"]), dev(s["e_occ"]), dev(s["e_vir"]), t, max_sweeps=3, hhl=True)
    assert e.value.code == -8
    eng.close()
