"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

FP64 results must match the FP64 oracle within 1e-12 relative Frobenius
error. Low-precision GEMMs are held to bounds derived from their arithmetic
(FP32: unit roundoff 6e-8 grown over sums of ~K terms; BF16x3: the two-term
split keeps ~16 mantissa bits per operand), stated next to each test.
"""
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
    from paper_2603_20912_amd import _lib
    _lib.load()
    return P


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def gpu_contract(P, s, t, prec="fp64", budget=0, tile=-1, alpha=1.0, beta=0.0, R0=None, config=None,
                 autotune=False):
    o, v, naux = s["o"], s["v"], s["naux"]
    eng = P.PPL(o, v, naux, prec=prec, hbm_budget=budget, tile_contract=tile)
    L = dev(s["L"])
    eng.build(L)
    if config is not None:
        eng.set_contract_config(*config)
    if autotune:
        eng.autotune(reps=1)
    R = dev(R0) if R0 is not None else torch.empty((o, o, v, v), dtype=torch.float64, device="cuda")
    eng.contract(dev(t), R, alpha, beta)
    torch.cuda.synchronize()
    out = R.cpu().numpy()
    info = eng.info
    eng.close()
    return out, info


# sizes span several GEMM tiles with ragged tails, plus the degenerate ends
CASES = [(5, 20, 60, 0), (1, 2, 1, 1), (2, 3, 5, 2), (3, 17, 23, 3), (4, 33, 70, 4), (6, 65, 40, 5),
         (9, 48, 130, 6), (2, 130, 17, 7)]


@pytest.mark.parametrize("o,v,naux,seed", CASES)
def test_contract_fp64_matches_oracle(P, o, v, naux, seed):
    say(f"contract fp64 o={o} v={v} naux={naux} seed={seed}")
    s = S.make_system(o, v, naux, seed)
    t = S.make_amplitudes(o, v, seed + 100)
    R, _ = gpu_contract(P, s, t)
    Rref = O.ppl(s["L"], o, t)
    assert rel(R, Rref) < 1e-12


def test_contract_mp2_amplitudes_c1(P):
    say("contract fp64 c1 MP2 amplitudes")
    s = S.make_system(5, 20, 60, 0)
    t = O.mp2_amplitudes(s["L"], 5, s["e_occ"], s["e_vir"])
    R, _ = gpu_contract(P, s, t)
    assert rel(R, O.ppl(s["L"], 5, t)) < 1e-12


def test_alpha_beta_accumulate(P):
    say("contract fp64 alpha/beta (4,21,30)")
    s = S.make_system(4, 21, 30, 11)
    t = S.make_amplitudes(4, 21, 12)
    R0 = np.random.default_rng(13).standard_normal((4, 4, 21, 21))
    R, _ = gpu_contract(P, s, t, alpha=-0.5, beta=2.0, R0=R0)
    ref = 2.0 * R0 - 0.5 * O.ppl(s["L"], 4, t)
    assert rel(R, ref) < 1e-12


@pytest.mark.parametrize("prec,bound", [("fp64", 1e-12), ("fp32", 2e-6), ("bf16x3", 4e-5), ("bf16x6", 2e-6)])
@pytest.mark.parametrize("tile", range(11))
def test_every_contraction_tile_and_split(P, tile, prec, bound):
    say(f"contract {prec} tile {tile} splits 1..8 and stream-K (7,37,130)")
    # K padded to 192: 12 FP64 / 6 FP32 chunks, so 8 slices are clamped to 6 for FP32 and BF16x3
    s = S.make_system(7, 37, 130, 20 + tile)
    t = S.make_amplitudes(7, 37, 30 + tile)
    Rref = O.ppl(s["L"], 7, t)
    first = None
    for sp in (1, 2, 3, 4, 6, 8, 0):
        # 0 = stream-K on the R+ GEMM; the R- GEMM takes another tile and K decomposition
        R, info = gpu_contract(P, s, t, prec=prec, config=(tile, sp, (tile + 1) % 11, (9 - sp) % 9))
        assert info["tile_contract"] == tile and info["splits_contract"] == sp
        assert rel(R, Rref) < bound
        if prec == "fp64":
            # different split counts change the summation order only
            if first is None:
                first = R
            assert rel(R, first) < 1e-14


def test_autotuned_contraction_matches(P):
    say("contract fp64 autotuned (12,90,200)")
    s = S.make_system(12, 90, 200, 60)
    t = S.make_amplitudes(12, 90, 61)
    R, info = gpu_contract(P, s, t, autotune=True)
    assert rel(R, O.ppl(s["L"], 12, t)) < 1e-12


def test_streaming_batches_match_resident(P):
    say("contract fp64 streaming (upper-triangle steps, U + U^T) vs resident (6,60,50), split-K")
    s = S.make_system(6, 60, 50, 40)
    t = S.make_amplitudes(6, 60, 41)
    R_res, i_res = gpu_contract(P, s, t, config=(5, 2, 0, 3))
    R_str, i_str = gpu_contract(P, s, t, budget=i_res["workspace_bytes"] // 3, config=(5, 2, 0, 3))
    assert i_res["resident"] == 1 and i_str["resident"] == 0 and i_str["n_batches"] > 1
    # V = U + U^T splits every sum into two GEMMs: equal up to rounding
    assert rel(R_str, R_res) < 1e-14
    assert rel(R_res, O.ppl(s["L"], 6, t)) < 1e-12


@pytest.mark.parametrize("prec,bound", [("fp32", 2e-6), ("bf16x3", 4e-5), ("bf16x6", 2e-6)])
def test_streaming_full_rows_low_precision(P, prec, bound):
    say(f"contract {prec} streaming (full rows) vs resident (6,60,50)")
    s = S.make_system(6, 60, 50, 42)
    t = S.make_amplitudes(6, 60, 43)
    R_res, i_res = gpu_contract(P, s, t, prec=prec)
    R_str, i_str = gpu_contract(P, s, t, prec=prec, budget=i_res["workspace_bytes"] // 3)
    assert i_res["resident"] == 1 and i_str["resident"] == 0 and i_str["n_batches"] > 1
    ref = O.ppl(s["L"], 6, t)
    assert rel(R_str, ref) < bound and rel(R_res, ref) < bound


@pytest.mark.parametrize("o,v,naux", [(1, 70, 20), (5, 130, 40), (9, 97, 61)])
def test_streaming_upper_triangle_steps(P, o, v, naux):
    say(f"contract fp64 streaming upper-triangle steps ({o},{v},{naux}), many steps")
    s = S.make_system(o, v, naux, 44)
    t = S.make_amplitudes(o, v, 45)
    eng = P.PPL(o, v, naux)
    budget = eng.info["workspace_bytes"] // 4
    eng.close()
    R, info = gpu_contract(P, s, t, budget=budget)
    assert info["resident"] == 0 and info["n_batches"] > 2
    assert info["flops_build"] == float(naux) * (info["p_plus"] ** 2 + v * (v + 1) * (2 * v + 1) // 6)
    assert rel(R, O.ppl(s["L"], o, t)) < 1e-12


def test_streaming_batches_stream_k(P):
    say("contract fp64 streaming vs resident (6,60,50), stream-K")
    s = S.make_system(6, 60, 50, 40)
    t = S.make_amplitudes(6, 60, 41)
    R_res, i_res = gpu_contract(P, s, t, config=(0, 0, 5, 0))
    R_str, i_str = gpu_contract(P, s, t, budget=i_res["workspace_bytes"] // 3, config=(0, 0, 5, 0))
    assert i_res["resident"] == 1 and i_str["resident"] == 0 and i_str["n_batches"] > 1
    # the K ranges of shared tiles follow each launch's partition, and V = U + U^T splits
    # the sums: equal up to rounding
    assert rel(R_str, R_res) < 1e-14
    assert rel(R_res, O.ppl(s["L"], 6, t)) < 1e-12
    # a repeated launch gives the same bits
    R_again, _ = gpu_contract(P, s, t, config=(0, 0, 5, 0))
    assert np.array_equal(R_res, R_again)


@pytest.mark.parametrize("prec,bound", [("fp32", 2e-6), ("bf16x3", 4e-5), ("bf16x6", 2e-6)])
def test_contract_low_precision(P, prec, bound):
    say(f"contract {prec} (8,60,180)")
    s = S.make_system(8, 60, 180, 50)
    t = O.mp2_amplitudes(s["L"], 8, s["e_occ"], s["e_vir"])
    R, _ = gpu_contract(P, s, t, prec=prec)
    err = rel(R, O.ppl(s["L"], 8, t))
    say(f"{prec} relative error {err:.3e}")
    assert err < bound


def test_iterate_fixed_sweeps_literal_c1(P):
    say("iterate fp64 10 literal sweeps c1")
    s = S.make_system(5, 20, 60, 0)
    eng = P.PPL(5, 20, 60)
    L, eo, ev = dev(s["L"]), dev(s["e_occ"]), dev(s["e_vir"])
    t = torch.zeros((5, 5, 20, 20), dtype=torch.float64, device="cuda")
    rep = eng.iterate(L, eo, ev, t, max_sweeps=10, tol=0.0, diverge_factor=0.0)
    eng.close()
    tref, hist, E = O.jacobi(s["L"], 5, s["e_occ"], s["e_vir"], max_sweeps=10, tol=0.0)
    assert rep["sweeps_fp64"] == 10 and rep["sweeps_lp"] == 0
    np.testing.assert_allclose(rep["history"], hist, rtol=1e-11)
    assert rel(t.cpu().numpy(), tref) < 1e-12
    assert abs(rep["energy"] - E) < 1e-12 * abs(E)
    V, D = O.mp2_parts(s["L"], 5, s["e_occ"], s["e_vir"])
    assert abs(rep["energy_start"] - O.energy(V, V / D)) < 1e-12 * abs(rep["energy_start"])


def test_iterate_converges_to_fixed_point(P):
    say("iterate fp64 to 1e-10, contractive c1")
    s = S.make_system(5, 20, 60, 0, "contractive")
    eng = P.PPL(5, 20, 60)
    t = torch.zeros((5, 5, 20, 20), dtype=torch.float64, device="cuda")
    rep = eng.iterate(dev(s["L"]), dev(s["e_occ"]), dev(s["e_vir"]), t, max_sweeps=200, tol=1e-10)
    eng.close()
    tstar = O.fixed_point(s["L"], 5, s["e_occ"], s["e_vir"])
    V, D = O.mp2_parts(s["L"], 5, s["e_occ"], s["e_vir"])
    assert rep["residual"] < 1e-10
    assert rel(t.cpu().numpy(), tstar) < 1e-8
    assert abs(rep["energy"] - O.energy(V, tstar)) < 1e-9


def test_literal_generator_diverges_and_is_reported(P):
    say("iterate fp64 divergence guard (6,40,120) literal")
    s = S.make_system(6, 40, 120, 3)
    eng = P.PPL(6, 40, 120)
    t = torch.zeros((6, 6, 40, 40), dtype=torch.float64, device="cuda")
    rep = eng.iterate(dev(s["L"]), dev(s["e_occ"]), dev(s["e_vir"]), t, max_sweeps=60, tol=1e-7,
                      diverge_factor=1e3, raise_on_status=False)
    eng.close()
    assert rep["rc"] == -6 and rep["status"] == -6


def test_c2_sampled_entries(P):
    say("contract fp64 c2 (20,200,600) sampled")
    o, v, naux = 20, 200, 600
    s = S.make_system(o, v, naux, 1)
    t = O.mp2_amplitudes(s["L"], o, s["e_occ"], s["e_vir"])
    R, info = gpu_contract(P, s, t)
    assert info["resident"] == 1
    rng = np.random.default_rng(7)
    idx = [tuple(int(x) for x in (rng.integers(o), rng.integers(o), rng.integers(v), rng.integers(v)))
           for _ in range(300)]
    idx += [(0, 0, 0, 0), (o - 1, o - 1, v - 1, v - 1), (0, o - 1, v - 1, 0), (3, 3, 5, 5)]
    ref = O.ppl_sampled(s["L"], o, t, idx)
    got = np.array([R[k] for k in idx])
    scale = np.abs(ref).max()
    assert np.abs(got - ref).max() < 1e-12 * scale
    # properties that hold at any size: pair symmetry of the result
    assert rel(R, R.transpose(1, 0, 3, 2)) < 1e-14


@pytest.mark.parametrize("prec,bound", [("fp64", 1e-12), ("fp32", 2e-6), ("bf16x3", 4e-5), ("bf16x6", 2e-6)])
@pytest.mark.parametrize("o,v,naux,scratch", [(7, 37, 130, 0), (5, 70, 45, 1 << 20), (3, 130, 33, 3 << 20)])
def test_upper_triangle_build_matches_full_rows(P, monkeypatch, prec, bound, o, v, naux, scratch):
    """Resident plans build the upper triangle of V+- and mirror it (one or several build
    steps); the result equals the full-row build and the oracle."""
    say(f"upper-triangle vs full-row build {prec} ({o},{v},{naux}), build scratch {scratch}")
    s = S.make_system(o, v, naux, 50)
    t = S.make_amplitudes(o, v, 51)
    out = {}
    for sym in ("1", "0"):
        monkeypatch.setenv("PPL_SYM_BUILD", sym)
        eng = P.PPL(o, v, naux, prec=prec, build_scratch=scratch)
        assert eng.info["resident"] == 1
        if scratch:
            assert eng.info["n_batches"] > 1
        eng.build(dev(s["L"]))
        out[sym] = eng.contract(dev(t)).cpu().numpy()
        eng.close()
    assert rel(out["1"], out["0"]) < (1e-14 if prec == "fp64" else bound / 10)
    assert rel(out["1"], O.ppl(s["L"], o, t)) < bound


def test_contract_only_plan(P):
    o, v, naux = 6, 40, 50
    say(f"contract-only plan ({o},{v},{naux})")
    s = S.make_system(o, v, naux, 60, "contractive")
    t = S.make_amplitudes(o, v, 61)
    eng = P.PPL(o, v, naux, contract_only=True)
    L = dev(s["L"])
    eng.build(L)
    R = eng.contract(dev(t)).cpu().numpy()
    assert rel(R, O.ppl(s["L"], o, t)) < 1e-12
    H = eng.hhl(L, dev(t)).cpu().numpy()
    assert rel(H, O.hhl(s["L"], o, t)) < 1e-12
    t2 = torch.zeros((o, o, v, v), dtype=torch.float64, device="cuda")
    with pytest.raises(P.PPLError) as e:
        eng.iterate(L, dev(s["e_occ"]), dev(s["e_vir"]), t2, max_sweeps=2)
    assert e.value.code == -7
    with pytest.raises(P.PPLError):
        eng.mp2(L, dev(s["e_occ"]), dev(s["e_vir"]))
    eng.close()


def test_asymmetric_cholesky_vectors_are_rejected(P):
    o, v, naux = 3, 20, 10
    say(f"build with asymmetric L ({o},{v},{naux}) is an argument error")
    s = S.make_system(o, v, naux, 70)
    L = s["L"].copy()
    L[2, o + 1, o + 5] += 1e-6 * np.abs(L).max()
    eng = P.PPL(o, v, naux)
    with pytest.raises(P.PPLError) as e:
        eng.build(dev(L))
    assert e.value.code == -1 and "symmetric" in str(e.value)
    eng.build(dev(s["L"]))                        # the symmetric vectors still build
    R = eng.contract(dev(S.make_amplitudes(o, v, 71))).cpu().numpy()
    assert rel(R, O.ppl(s["L"], o, S.make_amplitudes(o, v, 71))) < 1e-12
    eng.close()


def test_autotune_writes_the_tune_cache(P, tmp_path):
    o, v, naux = 5, 40, 30
    say(f"autotune with a tune cache ({o},{v},{naux})")
    s = S.make_system(o, v, naux, 80)
    path = tmp_path / "tune.txt"
    eng = P.PPL(o, v, naux, tune_cache=str(path))
    eng.build(dev(s["L"]))
    eng.contract(dev(S.make_amplitudes(o, v, 81)))
    eng.autotune(reps=1)
    cfg = eng.contract_config()
    eng.close()
    line = path.read_text().strip().splitlines()[-1].split()
    assert line[:5] == ["ppl-tune", "1", "0", str(o), str(v)] and tuple(int(x) for x in line[5:]) == cfg
    # a new plan of the shape starts from the tuned configuration
    eng2 = P.PPL(o, v, naux, tune_cache=str(path))
    assert eng2.contract_config() == cfg
    eng2.close()
