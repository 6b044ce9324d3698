"""GPU tests of the learned start: gradients and the Adam update of the
project's FP32 training kernels against the FP64 reference, the BF16-MFMA
inference against the reference forward pass, the MP2 amplitudes, and a small
end-to-end gain measurement on held-out instances."""
import sys

import numpy as np
import pytest

import oracle as O
from oracle import mlp_oracle as M
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


def dev(x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda")


def test_mp2_amplitudes_and_energy(P):
    say("ppl_mp2 (6,30,90)")
    s = S.make_system(6, 30, 90, 3)
    eng = P.PPL(6, 30, 90)
    t, e = eng.mp2(dev(s["L"]), dev(s["e_occ"]), dev(s["e_vir"]))
    V, D = O.mp2_parts(s["L"], 6, s["e_occ"], s["e_vir"])
    tref = V / D
    assert np.linalg.norm(t.cpu().numpy() - tref) / np.linalg.norm(tref) < 1e-12
    assert abs(e - O.energy(V, tref)) < 1e-12 * abs(e)
    eng.close()


@pytest.mark.parametrize("n", [1000, 4096])
def test_gradient_matches_reference(P, n):
    say(f"mlp gradient n={n}")
    p = M.init_params(128, seed=7)
    rng = np.random.default_rng(8)
    X = rng.standard_normal((n, 4)) * np.array([1.0, 3.0, 1.0, 2.0])
    Y = rng.standard_normal(n) * 0.3
    mlp = P.MLP(max_batch=8192)
    mlp.set_params(M.flatten(p).astype(np.float32))
    # the reference sees exactly the FP32-rounded inputs and parameters the kernels see
    p32 = M.unflatten(M.flatten(p).astype(np.float32).astype(np.float64), 128)
    X32 = X.astype(np.float32).astype(np.float64)
    Y32 = Y.astype(np.float32).astype(np.float64)
    g, loss = mlp.grad(dev(X, torch.float32), dev(Y, torch.float32))
    gref = M.flatten(M.grad(p32, X32, Y32))
    lref = M.loss(p32, X32, Y32)
    assert abs(loss - lref) < 1e-5 * abs(lref)
    off = 0
    for k in M.PARAM_ORDER:
        sz = p32[k].size
        a, b = g[off:off + sz].astype(np.float64), gref[off:off + sz]
        err = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        say(f"  grad {k}: rel err {err:.2e}")
        assert err < 1e-4, k
        off += sz
    mlp.close()


def test_adam_update_matches_reference(P):
    say("mlp adam step")
    p = M.init_params(128, seed=9)
    rng = np.random.default_rng(10)
    X = rng.standard_normal((512, 4))
    Y = rng.standard_normal(512)
    mlp = P.MLP(max_batch=1024)
    flat32 = M.flatten(p).astype(np.float32)
    mlp.set_params(flat32)
    g, _ = mlp.grad(dev(X, torch.float32), dev(Y, torch.float32))
    mlp.train_step(dev(X, torch.float32), dev(Y, torch.float32), lr=1e-3)
    got = mlp.get_params().astype(np.float64)
    q = M.unflatten(flat32.astype(np.float64), 128)
    M.adam_step(q, M.unflatten(g.astype(np.float64), 128), {}, lr=1e-3)
    ref = M.flatten(q)
    assert np.max(np.abs(got - ref)) < 1e-6
    mlp.close()


def test_training_reduces_loss(P):
    say("mlp training on a smooth target")
    rng = np.random.default_rng(11)
    X = rng.uniform(-2, 2, size=(8192, 4))
    Y = np.sin(X[:, 0]) * 0.5 + 0.2 * X[:, 1] * X[:, 2] - 0.1 * X[:, 3]
    mlp = P.MLP(max_batch=8192, seed=3)
    Xd, Yd = dev(X, torch.float32), dev(Y, torch.float32)
    _, l0 = mlp.grad(Xd, Yd)
    for _ in range(400):
        mlp.train_step(Xd, Yd, lr=3e-3)
    _, l1 = mlp.grad(Xd, Yd)
    say(f"  loss {l0:.4e} -> {l1:.4e}")
    assert l1 < 0.05 * l0
    mlp.close()


def test_guess_matches_reference_forward(P):
    say("mlp guess (BF16 MFMA) vs reference forward (5,21,63)")
    o, v, naux = 5, 21, 63
    s = S.make_system(o, v, naux, 12, "contractive")
    p = M.init_params(128, seed=13)
    mlp = P.MLP(max_batch=1024)
    mlp.set_params(M.flatten(p).astype(np.float32))
    eng = P.PPL(o, v, naux)
    eo, ev = dev(s["e_occ"]), dev(s["e_vir"])
    tm, _ = eng.mp2(dev(s["L"]), eo, ev)
    tg = mlp.guess(eng, tm, eo, ev)
    torch.cuda.synchronize()
    tm_h, tg_h = tm.cpu().numpy(), tg.cpu().numpy()
    X, sigma = M.features(tm_h, s["e_occ"], s["e_vir"])
    fref, _ = M.forward(p, X)
    fgot = ((tg_h - tm_h) / sigma).reshape(-1)
    # BF16 operands of the hidden layer: relative rounding 2^-8 per operand, summed over 128 terms
    err = np.max(np.abs(fgot - fref))
    say(f"  max |f_gpu - f_ref| = {err:.3e} (max |f| = {np.abs(fref).max():.3e})")
    assert err < 2e-2 * (1.0 + np.abs(fref).max())
    # every entry written and the guess is pair-symmetric
    assert np.isfinite(tg_h).all()
    assert np.array_equal(tg_h, tg_h.transpose(1, 0, 3, 2))
    eng.close()
    mlp.close()


def test_samples_match_reference_features(P):
    say("mlp samples (4,15,45)")
    o, v, naux = 4, 15, 45
    s = S.make_system(o, v, naux, 14, "contractive")
    eng = P.PPL(o, v, naux)
    eo, ev = dev(s["e_occ"]), dev(s["e_vir"])
    tm, _ = eng.mp2(dev(s["L"]), eo, ev)
    tstar = tm * 1.1
    sigma = P.ppl_mlp_sigma(eng.plan, tm)
    idx = torch.arange(0, o * o * v * v, 7, dtype=torch.int64, device="cuda")
    X = torch.empty((idx.numel(), 4), dtype=torch.float32, device="cuda")
    Y = torch.empty((idx.numel(),), dtype=torch.float32, device="cuda")
    P.ppl_mlp_samples(eng.plan, tm, tstar, eo, ev, sigma, idx, X, Y)
    Xr, sr = M.features(tm.cpu().numpy(), s["e_occ"], s["e_vir"])
    assert abs(sigma - sr) < 1e-14 * sr
    ii = idx.cpu().numpy()
    np.testing.assert_allclose(X.cpu().numpy(), Xr[ii], rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(Y.cpu().numpy(), 0.1 * tm.cpu().numpy().reshape(-1)[ii] / sr, rtol=1e-5, atol=1e-7)
    eng.close()


def test_learned_start_gain_small(P):
    """Train on converged amplitudes of small instances, measure on held-out ones."""
    from paper_2603_20912_amd import learned as Lr
    say("learned start: train on 10 small instances, evaluate on 3 held-out")
    gen = torch.Generator().manual_seed(0)
    shapes = S.training_shapes(10, seed=21, o_range=(4, 8), v_range=(16, 32))
    Xs, Ys = [], []
    for sh in shapes:
        sysd = S.make_system(sh["o"], sh["v"], sh["naux"], sh["seed"], "contractive")
        inst = Lr.converge(sysd, tol=1e-9)
        say(f"  train instance {sh}: sweeps {inst['report']['sweeps_fp64']} r {inst['report']['residual']:.1e}")
        X, Y = Lr.sample(inst, 20000, gen)
        Xs.append(X)
        Ys.append(Y)
        inst["eng"].close()
    X, Y = torch.cat(Xs), torch.cat(Ys)
    mlp = P.MLP(max_batch=4096, seed=1)
    hist = Lr.train(mlp, X, Y, steps=600, batch=4096, lr=2e-3, log_every=100)
    say(f"  training loss {hist[0][1]:.3e} -> {hist[-1][1]:.3e}")
    assert hist[-1][1] < hist[0][1]
    ratios, sw = [], []
    for k in range(3):
        sysd = S.make_system(8, 32, 96, 3000 + k, "contractive")
        inst = Lr.converge(sysd, tol=1e-11, max_sweeps=1000)
        tg = mlp.guess(inst["eng"], inst["t_mp2"], inst["d"]["e_occ"], inst["d"]["e_vir"], inst["sigma"])
        e_l = torch.linalg.norm(tg - inst["t_star"]).item()
        e_m = torch.linalg.norm(inst["t_mp2"] - inst["t_star"]).item()
        ratios.append(e_m / e_l)
        r_m, _ = Lr.time_to_tol(sysd, "mp2", tol=1e-7)
        r_l, _ = Lr.time_to_tol(sysd, "learned", mlp=mlp, tol=1e-7)
        r_c, _ = Lr.time_to_tol(sysd, "checked", mlp=mlp, tol=1e-7)
        sw.append((r_m["sweeps"], r_l["sweeps"], r_c["sweeps"], r_c["restarted_mp2"]))
        inst["eng"].close()
    say(f"  start-error reduction ||t_MP2-t*|| / ||t_guess-t*||: {[round(r, 3) for r in ratios]}")
    say(f"  sweeps to 1e-7 (mp2, learned, checked, restarted): {sw}")
    # the guess must be closer to the converged amplitudes than the first-order ones
    assert min(ratios) > 1.0
    # the learned start never needs more sweeps than the plain start
    assert all(l <= m for m, l, _, _ in sw)
    mlp.close()


@pytest.mark.parametrize("kind", ["nan", "inf", "worse"])
def test_checked_start_falls_back_to_mp2(P, kind):
    """A checked start whose guess holds a NaN or Inf is rejected before any sweep, and a
    finite guess with a larger first residual is rejected after its first sweep; either
    way the iteration continues from the MP2 amplitudes and ends where the MP2 start ends."""
    o, v, naux = 6, 30, 90
    say(f"checked start with a {kind} guess ({o},{v},{naux})")
    s = S.make_system(o, v, naux, 41, "contractive")
    L, eo, ev = dev(s["L"]), dev(s["e_occ"]), dev(s["e_vir"])
    eng = P.PPL(o, v, naux)
    t_ref = torch.empty((o, o, v, v), dtype=torch.float64, device="cuda")
    rep_ref = eng.iterate(L, eo, ev, t_ref, max_sweeps=200, tol=1e-10)
    tm, _ = eng.mp2(L, eo, ev)
    g = tm.clone()
    if kind == "nan":
        g[1, 2, 3, 4] = float("nan")
        g[2, 1, 4, 3] = float("nan")
    elif kind == "inf":
        g[0, 0, 5, 5] = float("inf")
    else:
        g.mul_(10.0)
    rep = eng.iterate(L, eo, ev, g, max_sweeps=200, tol=1e-10, start="checked")
    eng.close()
    assert rep["restarted_mp2"] == 1 and rep["status"] == 0
    assert rep["residual"] < 1e-10
    assert torch.isfinite(g).all().item()
    # the same MP2 sweeps as the plain start (the rejected guess adds its one sweep)
    extra = 0 if kind in ("nan", "inf") else 1
    assert rep["sweeps_fp64"] == rep_ref["sweeps_fp64"] + extra
    assert rel(g.cpu().numpy(), t_ref.cpu().numpy()) < 1e-14
    assert abs(rep["energy"] - rep_ref["energy"]) < 1e-13 * abs(rep_ref["energy"])
    if kind in ("nan", "inf"):
        assert abs(rep["energy_start"] - rep_ref["energy_start"]) < 1e-14 * abs(rep_ref["energy_start"])


def test_committed_weights_gain_on_held_out_instance(P):
    """The committed network (weights/mlp_start.f32) on one held-out (30, 300, 900)
    instance of the contractive generator (seed 3000, outside the training seeds): from its
    guess the FP64 iteration reaches 1e-7 in fewer sweeps than from the first-order
    amplitudes (24 against 30 when the weights were committed), at the same fixed point."""
    import os
    from paper_2603_20912_amd import learned as Lr
    weights = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                           "paper_2603_20912_amd", "weights", "mlp_start.f32")
    say("committed weights: held-out (30,300,900) seed 3000, FP64 sweeps to 1e-7, MP2 vs learned")
    sysd = S.make_system(30, 300, 900, 3000, "contractive")
    mlp = P.MLP(max_batch=1024)
    mlp.set_params(np.fromfile(weights, dtype="<f4"))
    r_m, t_m = Lr.time_to_tol(sysd, "mp2", tol=1e-7)
    r_l, t_l = Lr.time_to_tol(sysd, "learned", mlp=mlp, tol=1e-7)
    mlp.close()
    say(f"  sweeps mp2 {r_m['sweeps']} ({r_m['seconds']:.2f} s), learned {r_l['sweeps']} ({r_l['seconds']:.2f} s); "
        f"E {r_m['energy']:.10f} vs {r_l['energy']:.10f}")
    assert r_m["status"] == 0 and r_l["status"] == 0
    assert r_l["sweeps"] <= r_m["sweeps"] - 3
    assert abs(r_m["energy"] - r_l["energy"]) < 1e-7 * abs(r_m["energy"])
    assert rel(t_l.cpu().numpy(), t_m.cpu().numpy()) < 1e-5
    del t_m, t_l
    torch.cuda.empty_cache()
