"""CPU tests of the host side of libppl: the library loads, exports every
symbol the header declares, and the planner's decisions, byte accounting and
error codes behave as documented. No kernel is launched here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ppl.h")


@pytest.fixture(scope="module")
def P():
    import paper_2603_20912_amd as P
    from paper_2603_20912_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libppl.so is not built (run python -m paper_2603_20912_amd.build)")
    _lib.load()
    return P


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\**\s*(ppl_[a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol(P):
    from paper_2603_20912_amd import _lib
    names = declared_functions()
    assert len(names) >= 10, names
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), f"libppl.so does not export {n}"
    # and the binding declares a prototype for each of them
    assert set(names) <= set(_lib.SIGNATURES), set(names) - set(_lib.SIGNATURES)


def plan_info(P, *args, **kw):
    kw.setdefault("stream", 0)
    h = P.ppl_plan(*args, **kw)
    try:
        return P.ppl_plan_query(h)
    finally:
        P.ppl_destroy(h)


def test_pair_counts_and_flops(P):
    for o, v, naux in [(5, 20, 60), (20, 200, 600), (1, 2, 1), (7, 33, 5)]:
        i = plan_info(P, o, v, naux, hbm_budget=1 << 40)
        assert i["p_plus"] == v * (v + 1) // 2 and i["p_minus"] == v * (v - 1) // 2
        assert i["n_plus"] == o * (o + 1) // 2 and i["n_minus"] == o * (o - 1) // 2
        # resident plans build the upper triangle of V+-: rows (a, c >= a) times the packed
        # column pairs (b <= d) with b >= a, sum_{w=1..v} w^2 (w + 1) / 2 products of 2 naux
        # flops each; counted here by brute force over the (row, column) pairs kept
        kept = sum(1 for a in range(v) for c in range(a, v) for b in range(a, v) for d in range(b, v)) \
            if v <= 33 else sum((v - a) ** 2 * (v - a + 1) // 2 for a in range(v))
        assert i["resident"] == 1 and i["flops_build"] == 2.0 * naux * kept
        assert i["flops_contract"] == 2.0 * (i["p_plus"] ** 2 * i["n_plus"] + i["p_minus"] ** 2 * i["n_minus"])


def test_resident_when_budget_allows(P):
    i = plan_info(P, 20, 200, 600, hbm_budget=64 << 30)
    assert i["resident"] == 1
    assert i["workspace_bytes"] <= 64 << 30
    # FP64 V+- of (20, 200, 600): P+ rows of ldp + P- rows of ldm doubles
    ldp = (20100 + 63) // 64 * 64
    ldm = (19900 + 63) // 64 * 64
    assert i["vpm_bytes"] == (20100 * ldp + 19900 * ldm) * 8
    assert i["workspace_bytes"] > i["vpm_bytes"]


def test_budget_forces_streaming_batches(P):
    i = plan_info(P, 20, 200, 600, hbm_budget=1 << 30)
    assert i["resident"] == 0 and i["n_batches"] > 1
    assert i["workspace_bytes"] <= 1 << 30
    # FP64 streaming steps build the upper triangle as well (contracted as U and U^T);
    # other precisions stream full rows (2 naux v^2 flops per pair a <= b)
    assert i["flops_build"] == 600.0 * (i["p_plus"] ** 2 + 200 * 201 * 401 // 6)
    f32 = plan_info(P, 20, 200, 600, prec="fp32", hbm_budget=1 << 30)
    assert f32["resident"] == 0 and f32["flops_build"] == 2.0 * 600 * 200 * 200 * f32["p_plus"]


def test_streaming_plan_of_the_largest_benchmark_shape(P):
    # (nocc, nvir, nvec) = (100, 700, 4000) of the contraction benchmark (Tab. xc-split):
    # V+- would take about 960 GB in FP64, so the plan streams row batches; the split-K
    # slices span one batch (all columns would need 79 GB more than the budget holds)
    bud = 186 << 30
    i = plan_info(P, 100, 700, 4000, hbm_budget=bud, build_scratch=64 << 30)
    assert i["resident"] == 0 and i["n_batches"] > 1
    assert i["workspace_bytes"] <= bud
    # the planner takes (nearly) the largest build step that fits: one more virtual row
    # per step (at most v pairs: V+- rows, build scratch, transposed block) would not fit
    v, ldp = 700, (700 * 701 // 2 + 63) // 64 * 64
    row = v * (2 * ldp * 8 + v * v * 8 + ldp * 8)
    assert i["workspace_bytes"] > bud - 3 * row
    # a smaller budget streams in smaller steps
    j = plan_info(P, 100, 700, 4000, hbm_budget=170 << 30, build_scratch=64 << 30)
    assert j["max_step_pairs"] < i["max_step_pairs"] and j["n_batches"] > i["n_batches"]


def test_tune_cache_entries(P, tmp_path):
    path = tmp_path / "tune.txt"
    path.write_text("# a comment\n"
                    "ppl-tune 1 0 20 200 5 3 7 2\n"
                    "garbage line\n"
                    "ppl-tune 1 1 20 200 2 2 2 2\n"       # FP32: another key
                    "ppl-tune 1 0 20 200 6 0 8 6\n"       # the last FP64 entry wins
                    "ppl-tune 1 0 20 200 99 1 0 1\n")     # out of range: skipped
    i = plan_info(P, 20, 200, 600, hbm_budget=1 << 40, tune_cache=str(path))
    assert (i["tile_contract"], i["splits_contract"], i["tile_contract_minus"], i["splits_contract_minus"]) == \
        (6, 0, 8, 6)
    j = plan_info(P, 20, 200, 600, prec="fp32", hbm_budget=1 << 40, tune_cache=str(path))
    assert (j["tile_contract"], j["splits_contract"]) == (2, 2)
    # no entry for the shape, a missing file, or an explicit tile: the planner's own choice
    base = plan_info(P, 20, 200, 600, hbm_budget=1 << 40)
    for kw in (dict(tune_cache=str(tmp_path / "missing.txt")), dict(tune_cache=str(path), tile_contract=1)):
        k = plan_info(P, 20, 200, 600, hbm_budget=1 << 40, **kw)
        if "tile_contract" in kw:
            assert k["tile_contract"] == 1
        else:
            assert k["tile_contract"] == base["tile_contract"] and k["splits_contract"] == base["splits_contract"]
    other = plan_info(P, 21, 200, 600, hbm_budget=1 << 40, tune_cache=str(path))
    assert other["tile_contract"] == plan_info(P, 21, 200, 600, hbm_budget=1 << 40)["tile_contract"]


def test_tune_cache_keeps_bf16x6_slices(P, tmp_path):
    # at (40,400,1200) the padded K of both contractions needs at least 7 BF16x6 slices of
    # at most 12288 elements: lines with stream-K or fewer slices are skipped, the last
    # valid line wins
    path = tmp_path / "tune.txt"
    path.write_text("ppl-tune 1 3 40 400 9 7 9 8\n"
                    "ppl-tune 1 3 40 400 9 0 9 8\n"        # stream-K on R+: skipped
                    "ppl-tune 1 3 40 400 9 8 9 3\n")       # 3 slices on R-: skipped
    i = plan_info(P, 40, 400, 1200, prec="bf16x6", hbm_budget=1 << 40, tune_cache=str(path))
    assert (i["tile_contract"], i["splits_contract"], i["tile_contract_minus"], i["splits_contract_minus"]) == \
        (9, 7, 9, 8)
    path.write_text("ppl-tune 1 3 40 400 9 2 9 2\n")
    base = plan_info(P, 40, 400, 1200, prec="bf16x6", hbm_budget=1 << 40)
    j = plan_info(P, 40, 400, 1200, prec="bf16x6", hbm_budget=1 << 40, tune_cache=str(path))
    assert j["splits_contract"] == base["splits_contract"] >= 7
    assert j["splits_contract_minus"] == base["splits_contract_minus"] >= 7


def test_contract_only_plans(P):
    full = plan_info(P, 100, 700, 4000, hbm_budget=186 << 30, build_scratch=64 << 30)
    lean = plan_info(P, 100, 700, 4000, hbm_budget=186 << 30, build_scratch=64 << 30, flags=1)
    # the iteration's buffers go to V+- rows: larger streaming steps, fewer of them
    assert lean["max_step_pairs"] > full["max_step_pairs"] and lean["n_batches"] < full["n_batches"]
    assert lean["flops_build"] == full["flops_build"]
    small = plan_info(P, 20, 200, 600, hbm_budget=1 << 40, flags=1)
    assert small["workspace_bytes"] < plan_info(P, 20, 200, 600, hbm_budget=1 << 40)["workspace_bytes"]
    with pytest.raises(P.PPLError) as e:
        plan_info(P, 20, 200, 600, hbm_budget=1 << 40, flags=4)
    assert e.value.code == -1


def test_diis_slots_in_the_workspace(P):
    o, v, naux = 20, 200, 600
    base = plan_info(P, o, v, naux, hbm_budget=64 << 30)
    d8 = plan_info(P, o, v, naux, hbm_budget=64 << 30, diis_max=8)
    ldp, ldm = (20100 + 63) // 64 * 64, (19900 + 63) // 64 * 64
    slot = (210 * ldp + 190 * ldm) * 8            # one packed FP64 S'/A' vector
    extra = d8["workspace_bytes"] - base["workspace_bytes"]
    assert 2 * 8 * slot <= extra <= 2 * 8 * slot + (1024 + 1) * 16 * 8 + 3 * 256
    for bad in (-1, 17):
        with pytest.raises(P.PPLError) as e:
            plan_info(P, o, v, naux, hbm_budget=64 << 30, diis_max=bad)
        assert e.value.code == -1


def test_budget_too_small_is_nomem(P):
    with pytest.raises(P.PPLError) as e:
        plan_info(P, 20, 200, 600, hbm_budget=1 << 20)
    assert e.value.code == -2


def test_bf16x6_keeps_its_k_slices_short(P):
    # BF16x6 accuracy is set by the length of its FP32 accumulations: the planner splits K
    # into slices of at most 12288 elements (P+ = 80200 at v = 400: 7 slices; P- = 79800: 7)
    for (o, v, naux), want in (((40, 400, 1200), 7), ((30, 300, 900), 4), ((10, 100, 300), 1)):
        i = plan_info(P, o, v, naux, prec="bf16x6", hbm_budget=280 << 30)
        assert i["splits_contract"] >= want and i["splits_contract_minus"] >= want
        f = plan_info(P, o, v, naux, prec="fp32", hbm_budget=280 << 30)
        assert f["splits_contract"] >= 1


def test_ring_scratch_and_argument_checks(P):
    # staged ov, oo, vv blocks, the (kj|bc) product and seven (o v) x pad(o v) FP64 matrices
    o, v, naux = 40, 400, 1200
    ov, ldk, ldx = o * v, (o * v + 63) // 64 * 64, (naux + 63) // 64 * 64
    need = P.ppl_ring_scratch_bytes(o, v, naux)
    assert need >= 7 * ov * ldk * 8 + (ov + o * o + v * v) * ldx * 8
    assert need < 18 << 30
    assert P.ppl_ring_scratch_bytes(0, 4, 5) == 0 and P.ppl_ring_scratch_bytes(2, 4, 0) == 0
    from paper_2603_20912_amd import _lib
    # argument errors are caught on the host, before any device work
    rc = _lib.load().ppl_ring(2, 4, 5, None, None, None, 1.0, 0.0, None, 0, None)
    assert rc == _lib.PPL_E_ARG


def test_ring_plan_reserves_its_buffers(P):
    from paper_2603_20912_amd import _lib
    o, v, naux = 10, 100, 300
    base = plan_info(P, o, v, naux, hbm_budget=64 << 30)
    ring = plan_info(P, o, v, naux, hbm_budget=64 << 30, flags=_lib.PPL_PLAN_RING)
    extra = ring["workspace_bytes"] - base["workspace_bytes"]
    assert extra >= P.ppl_ring_scratch_bytes(o, v, naux) + 2 * o * o * v * v * 8
    assert extra < P.ppl_ring_scratch_bytes(o, v, naux) + 2 * o * o * v * v * 8 + (1 << 20)
    with pytest.raises(_lib.PPLError) as e:
        plan_info(P, o, v, naux, hbm_budget=64 << 30, flags=_lib.PPL_PLAN_RING | _lib.PPL_PLAN_CONTRACT_ONLY)
    assert e.value.code == _lib.PPL_E_ARG


def test_mixed_precision_keeps_both_copies(P):
    f64 = plan_info(P, 40, 400, 1200, prec="fp64", hbm_budget=280 << 30)
    mix = plan_info(P, 40, 400, 1200, prec="bf16x3", keep_fp64=True, hbm_budget=280 << 30)
    lp = plan_info(P, 40, 400, 1200, prec="bf16x3", keep_fp64=False, hbm_budget=280 << 30)
    assert mix["vpm_bytes"] == f64["vpm_bytes"] + lp["vpm_bytes"]
    assert lp["vpm_bytes"] * 2 == f64["vpm_bytes"]      # hi + lo bf16 planes = 4 bytes per element
    assert mix["workspace_bytes"] < 280 << 30 and mix["resident"] == 1
    x6 = plan_info(P, 40, 400, 1200, prec="bf16x6", keep_fp64=False, hbm_budget=280 << 30)
    x6mix = plan_info(P, 40, 400, 1200, prec="bf16x6", keep_fp64=True, hbm_budget=280 << 30)
    assert x6["vpm_bytes"] * 4 == f64["vpm_bytes"] * 3     # hi, mid and lo bf16 planes: 6 bytes
    assert x6mix["vpm_bytes"] == f64["vpm_bytes"] + x6["vpm_bytes"]
    assert x6mix["resident"] == 1 and x6mix["workspace_bytes"] < 280 << 30


@pytest.mark.parametrize("args,code", [
    (dict(o=0, v=10, naux=5), -1), (dict(o=2, v=1, naux=5), -1), (dict(o=2, v=10, naux=0), -1),
    (dict(o=2, v=10, naux=5, prec=7), -1), (dict(o=2, v=10, naux=5, tile_contract=99), -1),
    (dict(o=2, v=40000, naux=5), -1),
])
def test_invalid_arguments(P, args, code):
    kw = dict(hbm_budget=1 << 30, stream=0)
    kw.update(args)
    with pytest.raises(P.PPLError) as e:
        h = P.ppl_plan(kw.pop("o"), kw.pop("v"), kw.pop("naux"), **kw)
        P.ppl_destroy(h)
    assert e.value.code == code


def test_calls_out_of_order_are_state_errors(P):
    from paper_2603_20912_amd import _lib
    lib = _lib.load()
    h = P.ppl_plan(3, 8, 6, hbm_budget=1 << 30, stream=0)
    try:
        # no workspace bound: every device entry point refuses before touching HIP
        assert lib.ppl_build_batch(h, ctypes.c_void_p(256), -1) == -7
        assert lib.ppl_contract(h, ctypes.c_void_p(256), ctypes.c_void_p(512), 1.0, 0.0) == -7
        assert "workspace" in P.ppl_last_error()
        assert lib.ppl_contract_tau(h, ctypes.c_void_p(256), ctypes.c_void_p(768), ctypes.c_void_p(512),
                                    1.0, 0.0) == -7
        assert lib.ppl_hhl(h, ctypes.c_void_p(1024), ctypes.c_void_p(256), ctypes.c_void_p(512), 1.0, 0.0) == -7
        # misaligned workspace is an argument error
        assert lib.ppl_bind_workspace(h, ctypes.c_void_p(300), 1 << 30) == -1
    finally:
        P.ppl_destroy(h)


def test_iteration_defaults(P):
    o = P.ppl_iter_opts_default()
    assert o.max_sweeps == 100 and o.tol == 1e-7 and o.min_fp64_sweeps == 2 and o.diis == 0 and o.hhl == 0
    assert o.start == 0 and abs(o.stagnation - 0.95) < 1e-15 and o.switch_tol == 0.0


def test_product_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2603_20912_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "ppl_oracle" not in txt, f


def test_batch_plan_accounting(P):
    import ppl_synth as S
    shapes = [(d["o"], d["v"], d["naux"]) for d in S.batched_shapes(32, seed=4)]
    h = P.ppl_batch_plan(shapes, "fp64", stream=0)
    try:
        total, n_items = P.ppl_batch_query(h)
    finally:
        P.ppl_batch_destroy(h)
    # every instance's resident V+- is inside the batch workspace
    vpm = 0
    for o, v, naux in shapes:
        i = plan_info(P, o, v, naux, hbm_budget=1 << 60, build_scratch=256 << 20)
        assert i["resident"] == 1
        vpm += i["vpm_bytes"]
    assert total > vpm and total < 288e9
    assert n_items == 0          # items are laid out after the build
    with pytest.raises(P.PPLError):
        P.ppl_batch_plan(shapes[:2], "bf16x3", stream=0)


def test_mlp_handle_without_device(P):
    from paper_2603_20912_amd import _lib
    lib = _lib.load()
    h = P.ppl_mlp_create(128, 4096, stream=0)
    try:
        assert P.ppl_mlp_param_count(h) == 128 * 4 + 128 + 128 * 128 + 128 + 128 + 1
        nbytes = P.ppl_mlp_workspace_bytes(h)
        assert nbytes >= 4 * 4 * P.ppl_mlp_param_count(h)
        # unbound workspace: state error, no device access
        assert lib.ppl_mlp_init(h, 0) == -7
    finally:
        P.ppl_mlp_destroy(h)
    bad = ctypes.c_void_p()
    assert lib.ppl_mlp_create(64, 1024, None, ctypes.byref(bad)) == -8


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_2603_20912_amd import _lib
    saved = _lib._lib
    _lib._lib = None
    try:
        with pytest.raises(RuntimeError, match="no CPU fallback"):
            _lib.load(str(tmp_path / "missing.so"))
    finally:
        _lib._lib = saved


@pytest.mark.parametrize("o,v,naux,prec,keep", [(10, 100, 300, "bf16x3", True), (10, 100, 300, "fp32", True),
                                                (6, 40, 120, "bf16x3", False), (40, 400, 1200, "bf16x3", True),
                                                (20, 200, 600, "fp64", False)])
def test_build_scratch_holds_the_widest_accumulator(P, o, v, naux, prec, keep):
    # a mixed plan builds an FP64 copy too: its scratch must hold 8-byte integrals
    i = plan_info(P, o, v, naux, prec=prec, keep_fp64=keep, hbm_budget=280 << 30)
    acc = 8 if (prec == "fp64" or keep) else 4
    assert i["build_scratch_bytes"] >= i["max_step_pairs"] * v * v * acc
    assert i["build_scratch_bytes"] >= (o * v) ** 2 * 8


def test_tile_dims_and_contract_config_range(P):
    from paper_2603_20912_amd import _lib
    n = P.ppl_tile_count()
    assert n == 11   # the GPU tests walk tiles 0 .. 10
    dims = [P.ppl_tile_dims(t) for t in range(n)]
    # MFMA blocks are 16 x 16 and contraction workgroups have four or eight waves
    assert all(bm % 16 == 0 and bn % 16 == 0 and th in (256, 512) for bm, bn, th in dims)
    for bad in (-1, n):
        with pytest.raises(_lib.PPLError) as e:
            P.ppl_tile_dims(bad)
        assert e.value.code == _lib.PPL_E_ARG
    plan = _lib.ppl_plan(5, 20, 60, hbm_budget=1 << 30, stream=False)
    try:
        for sp in (0, 1, 8):   # 0 = stream-K
            _lib.ppl_set_contract_config(plan, 0, sp, 1, sp)
            info = _lib.ppl_plan_query(plan)
            assert info["splits_contract"] == sp and info["splits_contract_minus"] == sp
        for sp in (-1, 9):
            with pytest.raises(_lib.PPLError) as e:
                _lib.ppl_set_contract_config(plan, 0, sp, 0, 1)
            assert e.value.code == _lib.PPL_E_ARG
    finally:
        _lib.ppl_destroy(plan)


def test_binding_rejects_bad_tensors_before_the_library(P):
    """The C ABI sees bare addresses: the binding checks dtype, shape, contiguity and device
    of every tensor against the documented layouts and raises ValueError first (CPU tensors
    of the right layout fail on the device check only)."""
    import numpy as np
    import torch
    o, v, naux = 3, 8, 6
    h = P.ppl_plan(o, v, naux, hbm_budget=1 << 30, stream=0)
    f64 = dict(dtype=torch.float64)
    good = torch.zeros((o, o, v, v), **f64)
    try:
        bad_amps = [(torch.zeros((o, o, v, v), dtype=torch.float32), "dtype"),
                    (torch.zeros((o, o, v, v + 1), **f64), "shape"),
                    (torch.zeros((o, o, v, v), **f64).transpose(2, 3), "contiguous"),
                    (good, "GPU"),
                    (np.zeros((o, o, v, v)), "torch.Tensor"),
                    (None, "required")]
        for bad, msg in bad_amps:
            with pytest.raises(ValueError, match=msg):
                P.ppl_contract(h, bad, good)
            with pytest.raises(ValueError, match=msg):
                P.ppl_contract(h, good, bad)
        n = o + v
        for L, msg in [(torch.zeros((naux, n, n + 1), **f64), "shape"), (torch.zeros((naux, n, n)), "dtype"),
                       (torch.zeros((naux, n, n), **f64), "GPU")]:
            with pytest.raises(ValueError, match=msg):
                P.ppl_build_batch(h, L)
            with pytest.raises(ValueError, match=msg):
                P.ppl_hhl(h, L, good, good)
        eo, ev = torch.zeros(o, **f64), torch.zeros(v, **f64)
        with pytest.raises(ValueError, match="e_occ.*shape"):
            P.ppl_mp2(h, torch.zeros((naux, n, n), **f64), torch.zeros(o + 1, **f64), ev, good)
        with pytest.raises(ValueError, match="e_vir.*dtype"):
            P.ppl_iterate(h, torch.zeros((naux, n, n), **f64), eo, torch.zeros(v), good)
        with pytest.raises(ValueError, match="t1.*shape"):
            P.ppl_contract_tau(h, good, torch.zeros((v, o), **f64), good)
    finally:
        P.ppl_destroy(h)
    # a destroyed plan is no longer known to the binding
    with pytest.raises(ValueError, match="unknown"):
        P.ppl_contract(h, good, good)
    # the ring terms take their sizes as arguments
    with pytest.raises(ValueError, match="R.*shape"):
        P.ppl_ring(o, v, naux, torch.zeros((naux, o + v, o + v), **f64), good, torch.zeros((o, o, v, 1), **f64),
                   torch.zeros(16, dtype=torch.uint8))
    # the learned start: X [n][4] and Y [n] in FP32, index vectors in int64
    m = P.ppl_mlp_create(128, 4096, stream=0)
    try:
        with pytest.raises(ValueError, match="X.*shape"):
            P.ppl_mlp_train_step(m, torch.zeros((10, 3)), torch.zeros(10), 1e-3)
        with pytest.raises(ValueError, match="Y.*dtype"):
            P.ppl_mlp_grad(m, torch.zeros((10, 4)), torch.zeros(10, dtype=torch.float64))
    finally:
        P.ppl_mlp_destroy(m)
    h = P.ppl_plan(o, v, naux, hbm_budget=1 << 30, stream=0)
    try:
        with pytest.raises(ValueError, match="idx.*dtype"):
            P.ppl_mlp_samples(h, good, None, eo, ev, 1.0, torch.zeros(5, dtype=torch.int32), torch.zeros((5, 4)))
    finally:
        P.ppl_destroy(h)
    # batched instances: one tensor per instance, each of its own instance's layout
    shapes = [(2, 6, 5), (3, 8, 6)]
    b = P.ppl_batch_plan(shapes, "fp64", stream=0)
    try:
        ts = [torch.zeros((2, 2, 6, 6), **f64), torch.zeros((3, 3, 8, 8), **f64)]
        with pytest.raises(ValueError, match="one per instance"):
            P.ppl_batch_contract(b, ts[:1], ts[:1])
        with pytest.raises(ValueError, match=r"t2\[1\].*shape"):
            P.ppl_batch_contract(b, [ts[0], ts[0]], ts)
        with pytest.raises(ValueError, match=r"L\[0\].*GPU"):
            P.ppl_batch_build(b, [torch.zeros((5, 8, 8), **f64), torch.zeros((6, 11, 11), **f64)])
    finally:
        P.ppl_batch_destroy(b)
