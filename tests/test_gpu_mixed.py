"""GPU tests of the mixed-precision path: single-evaluation errors of the FP32
and BF16x3 GEMMs against the emulation of their rounding points, and the
mixed iteration (low-precision sweeps, then FP64 refinement) converging to the
FP64 fixed point within the stated bounds (amplitudes 1e-6 relative, energy
1e-6 Eh)."""
import sys

import numpy as np
import pytest

import oracle as O
from oracle import precision_oracle as Pr
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


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16x6"])
def test_single_evaluation_error_matches_emulation(P, prec):
    o, v, naux = 6, 36, 108
    say(f"{prec} single R vs emulation ({o},{v},{naux})")
    s = S.make_system(o, v, naux, 31)
    t = O.mp2_amplitudes(s["L"], o, s["e_occ"], s["e_vir"])
    Rref = O.ppl(s["L"], o, t)
    eng = P.PPL(o, v, naux, prec=prec)
    eng.build(dev(s["L"]))
    R = eng.contract(dev(t)).cpu().numpy()
    eng.close()
    e_gpu = rel(R, Rref)
    e_emu = rel(Pr.ppl_lowprec(s["L"], o, t, prec), Rref)
    say(f"  relative error gpu {e_gpu:.3e}, emulated {e_emu:.3e}")
    # same rounding points; FP32 accumulation order adds at most a small factor
    assert e_gpu < 3.0 * e_emu + 1e-7
    assert e_gpu > 0.2 * e_emu


@pytest.mark.parametrize("prec", ["bf16x3", "fp32", "bf16x6"])
def test_mixed_iteration_reaches_fp64_fixed_point(P, prec):
    o, v, naux = 10, 100, 300
    say(f"mixed {prec} -> fp64 iteration to 1e-7 ({o},{v},{naux}) contractive")
    s = S.make_system(o, v, naux, 1, "contractive")
    L, eo, ev = dev(s["L"]), dev(s["e_occ"]), dev(s["e_vir"])
    eng = P.PPL(o, v, naux, prec=prec, keep_fp64=True)
    t = torch.zeros((o, o, v, v), dtype=torch.float64, device="cuda")
    rep = eng.iterate(L, eo, ev, t, max_sweeps=200, tol=1e-7)
    eng.close()
    say(f"  sweeps lp {rep['sweeps_lp']} fp64 {rep['sweeps_fp64']}, residual {rep['residual']:.2e}, "
        f"E {rep['energy']:.10f}")
    assert rep["status"] == 0 and rep["residual"] < 1e-7
    assert rep["sweeps_lp"] > 0 and rep["sweeps_fp64"] >= 2
    tstar, hist, Estar = O.jacobi(s["L"], o, s["e_occ"], s["e_vir"], max_sweeps=200, tol=1e-11)
    err_t = rel(t.cpu().numpy(), tstar)
    say(f"  |t - t*|/|t*| = {err_t:.2e}, |E - E*| = {abs(rep['energy'] - Estar):.2e} (E* = {Estar:.10f})")
    assert err_t < 1e-6
    assert abs(rep["energy"] - Estar) < 1e-6


def test_low_precision_alone_stalls_at_its_floor(P):
    o, v, naux = 6, 40, 120
    say(f"bf16x3 without FP64 refinement ({o},{v},{naux})")
    s = S.make_system(o, v, naux, 2, "contractive")
    eng = P.PPL(o, v, naux, prec="bf16x3", keep_fp64=False)
    t = torch.zeros((o, o, v, v), dtype=torch.float64, device="cuda")
    rep = eng.iterate(dev(s["L"]), dev(s["e_occ"]), dev(s["e_vir"]), t, max_sweeps=80, tol=1e-12,
                      raise_on_status=False)
    eng.close()
    say(f"  floor residual {rep['residual']:.2e} after {rep['sweeps_lp']} sweeps, status {rep['status']}")
    assert rep["status"] == -5 and rep["sweeps_fp64"] == 0
    assert 1e-12 < rep["residual"] < 1e-4
