"""The ring terms without allocation (ppl_ring_static) against ppl_ring with a caller
scratch: two calls in a row on the same GPU, the second with a smaller input, so that
the second runs on the static scratch the first one left behind."""
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


def test_ring_static_matches_ring_on_two_calls(P):
    torch.cuda.synchronize()
    for k, (o, v, naux, beta) in enumerate([(7, 52, 150, 0.0), (3, 17, 40, 0.5)]):
        need = P.ppl_ring_scratch_bytes(o, v, naux)
        say(f"ring_static call {k}: ({o},{v},{naux}) needs {need} B of {P._lib.PPL_RING_STATIC_BYTES}")
        assert 0 < need <= P._lib.PPL_RING_STATIC_BYTES
        s = S.make_system(o, v, naux, 60 + k)
        t = S.make_amplitudes(o, v, 70 + k)
        R0 = S.make_amplitudes(o, v, 80 + k)
        L, td = torch.from_numpy(s["L"]).cuda(), torch.from_numpy(t).cuda()
        R_ref = torch.from_numpy(R0).cuda()
        R_st = R_ref.clone()
        scratch = torch.empty(need, dtype=torch.uint8, device="cuda")
        P.ppl_ring(o, v, naux, L, td, R_ref, scratch, 1.5, beta)
        P.ppl_ring_static(o, v, naux, L, td, R_st, 1.5, beta)
        torch.cuda.synchronize()
        a, b = R_st.cpu().numpy(), R_ref.cpu().numpy()
        # the same kernels on the same inputs: the same bits
        assert np.array_equal(a, b), rel(a, b)
        ref = beta * R0 + 1.5 * O.ring(s["L"], o, t)
        err = rel(a, ref)
        say(f"  relative error against the oracle {err:.2e}")
        assert err < 1e-12


def test_ring_static_rejects_sizes_beyond_its_scratch(P):
    o, v, naux = 12, 120, 360
    assert P.ppl_ring_scratch_bytes(o, v, naux) > P._lib.PPL_RING_STATIC_BYTES
    n = o + v
    L = torch.zeros((naux, n, n), dtype=torch.float64, device="cuda")
    t = torch.zeros((o, o, v, v), dtype=torch.float64, device="cuda")
    R = torch.zeros_like(t)
    with pytest.raises(P.PPLError) as e:
        P.ppl_ring_static(o, v, naux, L, t, R)
    assert e.value.code == -1 and "static scratch" in str(e.value)
    # R aliasing t2 is an argument error, as for ppl_ring
    ts = torch.zeros((2, 2, 5, 5), dtype=torch.float64, device="cuda")
    with pytest.raises(P.PPLError) as e:
        P.ppl_ring_static(2, 5, 4, torch.zeros((4, 7, 7), dtype=torch.float64, device="cuda"), ts, ts)
    assert e.value.code == -1
