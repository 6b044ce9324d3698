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
