"""GPU tests of the CCSD terms next to the ladder: the ladder with singles,
PPL(t2 + t1 t1) (ppl_contract_tau), and the hole-hole ladder
sum_kl (ki|lj) t_kl^ab (ppl_hhl), against the oracle element by element."""
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


@pytest.mark.parametrize("o,v,naux,prec,bound", [(7, 37, 130, "fp64", 1e-12), (3, 20, 17, "fp64", 1e-12),
                                                 (7, 37, 130, "fp32", 2e-6), (7, 37, 130, "bf16x3", 4e-5),
                                                 (7, 37, 130, "bf16x6", 2e-6)])
def test_contract_tau_matches_oracle(P, o, v, naux, prec, bound):
    say(f"contract_tau {prec} ({o},{v},{naux})")
    s = S.make_system(o, v, naux, 21)
    t2 = S.make_amplitudes(o, v, 22)
    t1 = 0.3 * np.random.default_rng(23).standard_normal((o, v))
    eng = P.PPL(o, v, naux, prec=prec)
    eng.build(dev(s["L"]))
    R = eng.contract(dev(t2), t1=dev(t1)).cpu().numpy()
    eng.close()
    ref = O.ppl_tau(s["L"], o, t2, t1)
    assert rel(R, ref) < bound
    # the singles really enter (the plain ladder differs by far more than the bound)
    assert rel(O.ppl(s["L"], o, t2), ref) > 1e3 * bound


@pytest.mark.parametrize("o,v,naux", [(1, 5, 6), (2, 9, 10), (7, 37, 130), (12, 60, 40), (20, 33, 70)])
def test_hhl_matches_oracle(P, o, v, naux):
    say(f"hhl fp64 ({o},{v},{naux})")
    s = S.make_system(o, v, naux, 31)
    t2 = S.make_amplitudes(o, v, 32)
    eng = P.PPL(o, v, naux)
    L = dev(s["L"])
    R = eng.hhl(L, dev(t2)).cpu().numpy()
    ref = O.hhl(s["L"], o, t2)
    assert rel(R, ref) < 1e-12
    # accumulate: R <- 0.5 R0 + 2 HHL
    R0 = np.random.default_rng(33).standard_normal(t2.shape)
    Rd = dev(R0)
    eng.hhl(L, dev(t2), Rd, alpha=2.0, beta=0.5)
    assert rel(Rd.cpu().numpy(), 0.5 * R0 + 2.0 * ref) < 1e-12
    eng.close()


def test_hhl_in_a_streaming_plan(P):
    o, v, naux = 6, 60, 50
    say(f"hhl fp64 streaming plan ({o},{v},{naux})")
    s = S.make_system(o, v, naux, 40)
    t2 = S.make_amplitudes(o, v, 41)
    res = P.PPL(o, v, naux)
    str_ = P.PPL(o, v, naux, hbm_budget=res.info["workspace_bytes"] // 3)
    assert str_.info["resident"] == 0
    L = dev(s["L"])
    R1 = res.hhl(L, dev(t2)).cpu().numpy()
    R2 = str_.hhl(L, dev(t2)).cpu().numpy()
    res.close()
    str_.close()
    assert np.array_equal(R1, R2)
    assert rel(R1, O.hhl(s["L"], o, t2)) < 1e-12


def test_hhl_in_chunks_of_virtual_pairs(P):
    # a contract-only plan with a small build scratch: the transposed operands of the
    # hole-hole ladder go through it in several chunks of virtual pairs
    o, v, naux = 60, 140, 30
    say(f"hhl fp64 ({o},{v},{naux}) in chunks of virtual pairs")
    s = S.make_system(o, v, naux, 34)
    t2 = S.make_amplitudes(o, v, 35)
    eng = P.PPL(o, v, naux, contract_only=True, build_scratch=1 << 20)
    L = dev(s["L"])
    R = eng.hhl(L, dev(t2)).cpu().numpy()
    eng.close()
    assert rel(R, O.hhl(s["L"], o, t2)) < 1e-12


@pytest.mark.parametrize("o,v,naux", [(7, 37, 130), (3, 20, 17), (1, 5, 3), (9, 70, 61)])
def test_ring_matches_oracle(P, o, v, naux):
    say(f"ring fp64 ({o},{v},{naux})")
    s = S.make_system(o, v, naux, 71)
    t = S.make_amplitudes(o, v, 72)
    R0 = np.random.default_rng(73).standard_normal((o, o, v, v))
    R = dev(R0.copy())
    P.ring(dev(s["L"]), dev(t), R, alpha=-0.5, beta=2.0)
    ref = 2.0 * R0 - 0.5 * O.ring(s["L"], o, t)
    got = R.cpu().numpy()
    assert rel(got, ref) < 1e-12
    # beta = 0 overwrites (R may hold anything, NaN included)
    Rn = torch.full((o, o, v, v), float("nan"), dtype=torch.float64, device="cuda")
    P.ring(dev(s["L"]), dev(t), Rn)
    assert rel(Rn.cpu().numpy(), O.ring(s["L"], o, t)) < 1e-12


def test_ring_rejects_small_scratch_and_aliasing(P):
    o, v, naux = 3, 20, 17
    say(f"ring argument checks ({o},{v},{naux})")
    s = S.make_system(o, v, naux, 74)
    L, t = dev(s["L"]), dev(S.make_amplitudes(o, v, 75))
    need = P.ppl_ring_scratch_bytes(o, v, naux)
    small = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(P.PPLError) as e:
        P.ring(L, t, torch.empty_like(t), scratch=small)
    assert e.value.code == -1
    with pytest.raises(P.PPLError):
        P.ring(L, t, t)


def test_ring_c3_sampled(P):
    o, v, naux = 40, 400, 1200
    say(f"ring fp64 ({o},{v},{naux}) sampled")
    s = S.make_system(o, v, naux, 2, "contractive")
    t = S.make_amplitudes(o, v, 3)
    R = P.ring(dev(s["L"]), dev(t))
    torch.cuda.synchronize()
    rng = np.random.default_rng(76)
    idx = [tuple(int(x) for x in (rng.integers(o), rng.integers(o), rng.integers(v), rng.integers(v)))
           for _ in range(12)] + [(0, 0, 0, 0), (o - 1, o - 1, v - 1, v - 1), (0, o - 1, v - 1, 0)]
    ref = np.array([O.ring_entry(s["L"], o, t, *k) for k in idx])
    got = np.array([R[k].item() for k in idx])
    err = np.abs(got - ref).max() / np.abs(ref).max()
    say(f"  max |R_gpu - R_oracle| / max |R| = {err:.2e}")
    assert err < 1e-12
    assert (torch.linalg.norm(R - R.permute(1, 0, 3, 2)) / torch.linalg.norm(R)).item() < 1e-14
    del R
    torch.cuda.empty_cache()


def test_iteration_with_ring_matches_oracle_sweep_by_sweep(P):
    """Plain FP64 sweeps of t = (V + PPL(t) + HHL(t) + RING(t)) / D against the oracle's,
    residual by residual, to r < 1e-7 (the contractive generator converges at this size)."""
    o, v, naux = 6, 40, 120
    say(f"iterate fp64 with hhl + ring ({o},{v},{naux}) contractive")
    s = S.make_system(o, v, naux, 1, "contractive")
    eng = P.PPL(o, v, naux, ring=True)
    t = torch.zeros((o, o, v, v), dtype=torch.float64, device="cuda")
    rep = eng.iterate(dev(s["L"]), dev(s["e_occ"]), dev(s["e_vir"]), t, max_sweeps=100, tol=1e-7, hhl=True,
                      ring=True)
    eng.close()
    tref, hist, E = O.jacobi(s["L"], o, s["e_occ"], s["e_vir"], max_sweeps=100, tol=1e-7, with_hhl=True,
                             with_ring=True)
    say(f"  sweeps {rep['sweeps_fp64']} (oracle {len(hist)}), residual {rep['residual']:.2e}")
    assert rep["status"] == 0 and rep["sweeps_fp64"] == len(hist)
    np.testing.assert_allclose(rep["history"], hist, rtol=1e-8)
    assert rel(t.cpu().numpy(), tref) < 1e-10
    assert abs(rep["energy"] - E) < 1e-10 * abs(E)


def test_diis_with_ring_reaches_the_dense_fixed_point(P):
    """At this tiny size the plain sweeps diverge with the ring terms; DIIS reaches the
    fixed point of the full operator, solved densely by the oracle."""
    o, v, naux = 2, 5, 8
    say(f"iterate fp64 diis 6 with hhl + ring ({o},{v},{naux})")
    s = S.make_system(o, v, naux, 12, "contractive")
    eng = P.PPL(o, v, naux, ring=True, diis_max=6)
    t = torch.zeros((o, o, v, v), dtype=torch.float64, device="cuda")
    rep = eng.iterate(dev(s["L"]), dev(s["e_occ"]), dev(s["e_vir"]), t, max_sweeps=200, tol=1e-11, hhl=True,
                      ring=True, diis=6)
    eng.close()
    tstar = O.fixed_point_terms(s["L"], o, s["e_occ"], s["e_vir"])
    assert rep["status"] == 0
    assert np.abs(t.cpu().numpy() - tstar).max() < 1e-9 * np.abs(tstar).max()


@pytest.mark.parametrize("prec,bound", [("bf16x3", 2e-5), ("fp32", 2e-6), ("bf16x6", 2e-6)])
def test_low_precision_ring_sweep_matches_oracle(P, prec, bound):
    """The first sweep of a mixed plan runs the ladder and the ring GEMMs in the low
    precision: its residual must equal the oracle's FP64 first-sweep residual to the
    level of the low-precision products (a wrong ring term would be off by O(1))."""
    o, v, naux = 6, 40, 120
    say(f"one {prec} sweep with hhl + ring ({o},{v},{naux}) against the oracle")
    s = S.make_system(o, v, naux, 1, "contractive")
    eng = P.PPL(o, v, naux, prec=prec, keep_fp64=True, ring=True)
    t = torch.zeros((o, o, v, v), dtype=torch.float64, device="cuda")
    rep = eng.iterate(dev(s["L"]), dev(s["e_occ"]), dev(s["e_vir"]), t, max_sweeps=1, tol=0.0, hhl=True,
                      ring=True, switch_tol=1e-30, stagnation=10.0)
    eng.close()
    assert rep["sweeps_lp"] == 1 and rep["sweeps_fp64"] == 0
    tref, hist, _ = O.jacobi(s["L"], o, s["e_occ"], s["e_vir"], max_sweeps=1, tol=0.0, with_hhl=True,
                             with_ring=True)
    err_r = abs(rep["history"][0] - hist[0]) / hist[0]
    err_t = rel(t.cpu().numpy(), tref)
    say(f"  residual {rep['history'][0]:.6e} vs {hist[0]:.6e} (rel {err_r:.1e}); amplitudes rel {err_t:.1e}")
    assert err_r < bound and err_t < bound


@pytest.mark.parametrize("prec", ["bf16x3", "fp32", "bf16x6"])
def test_mixed_iteration_with_ring(P, prec):
    o, v, naux = 10, 100, 300
    say(f"mixed {prec} -> fp64 with hhl + ring and diis 8 to 1e-7 ({o},{v},{naux})")
    s = S.make_system(o, v, naux, 1, "contractive")
    eng = P.PPL(o, v, naux, prec=prec, keep_fp64=True, ring=True, diis_max=8)
    t = torch.zeros((o, o, v, v), dtype=torch.float64, device="cuda")
    rep = eng.iterate(dev(s["L"]), dev(s["e_occ"]), dev(s["e_vir"]), t, max_sweeps=200, tol=1e-7, hhl=True,
                      ring=True, diis=8)
    eng.close()
    assert rep["status"] == 0 and rep["residual"] < 1e-7 and rep["sweeps_lp"] > 0 and rep["sweeps_fp64"] >= 2
    tstar, _, Estar = O.jacobi_diis(s["L"], o, s["e_occ"], s["e_vir"], m=8, max_sweeps=200, tol=1e-10,
                                    with_hhl=True, with_ring=True)
    assert rel(t.cpu().numpy(), tstar) < 1e-6
    assert abs(rep["energy"] - Estar) < 1e-6


def test_ring_iteration_needs_a_ring_plan(P):
    o, v, naux = 3, 12, 20
    say(f"iterate with ring on a plan without PPL_PLAN_RING ({o},{v},{naux})")
    s = S.make_system(o, v, naux, 5, "contractive")
    eng = P.PPL(o, v, naux)
    t = torch.zeros((o, o, v, v), dtype=torch.float64, device="cuda")
    with pytest.raises(P.PPLError) as e:
        eng.iterate(dev(s["L"]), dev(s["e_occ"]), dev(s["e_vir"]), t, max_sweeps=3, ring=True)
    assert e.value.code == -7
    eng.close()
