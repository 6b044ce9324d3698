#!/usr/bin/env python3
"""Benchmark of the particle-particle ladder (PPL) hot path on one MI355X.

One step = the whole FP64 hot path at (o, v, naux) = (20, 200, 600) with the
literal input generator (seed 1), all inputs already resident in HBM:
  * (ia|jb) and the MP2 start in the packed pair space,
  * the V+- integral build from the Cholesky vectors (one build),
  * 10 Jacobi sweeps t <- (V + PPL(t)) / D (one contraction + FP64 update,
    residual and energy each),
  * one more PPL evaluation R = PPL(t) of the final amplitudes, unpacked to
    the caller's [o][o][v][v] array.
value = useful flops of the pair method (one build of the upper triangle of V+-
over packed column pairs, naux (P+^2 + v(v+1)(2v+1)/6), + 11 contractions) / step time. The dominant kernel is the R+ contraction GEMM; its roofline entry uses
HIP-event timings of its launches inside the timed region.

The same JSON line carries the metric's second half under "time_to_residual": wall time
to an amplitude residual of 1e-7 at (40, 400, 1200) for plain FP64 and for BF16x3 sweeps
refined in FP64 (MP2 and learned starts), without and with DIIS, with like-for-like
speed-ups; and under "cpu_baseline" the oracle's timing on the host cores (median of 5
after one untimed run) and its sampled residual of the mixed + learned + DIIS result.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-c3]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PPL TFLOP/s + % MFMA peak; time-to-converged residual, FP64 vs mixed+learned"
PEAK_FP64_TFLOPS = 78.6        # MI355X dense FP64 matrix peak
O_, V_, NAUX_, SEED_ = 20, 200, 600, 1
SWEEPS = 10


def nominal(o, v, naux, upper=True):
    """Useful flops of the pair method. FP64 plans build the upper triangle of V+-
    (rows (a, c >= a), columns the packed pairs (b <= d) with b >= a: 2 naux (v - a)^2
    (v - a + 1) / 2 per virtual a, i.e. naux (P+^2 + v(v+1)(2v+1)/6)); streaming plans of
    the other precisions build every row in full (2 naux v^2 P+)."""
    Pp, Pm = v * (v + 1) // 2, v * (v - 1) // 2
    Np, Nm = o * (o + 1) // 2, o * (o - 1) // 2
    sq = v * (v + 1) * (2 * v + 1) // 6
    build = float(naux) * (Pp * Pp + sq) if upper else 2.0 * naux * v * v * Pp
    return {"build": build, "contract": 2.0 * (Pp * Pp * Np + Pm * Pm * Nm),
            "contract_plus": 2.0 * Pp * Pp * Np, "contract_minus": 2.0 * Pm * Pm * Nm}


def host_description():
    """nproc, CPU model and the BLAS numpy calls, recorded with every oracle timing."""
    import numpy as np
    model = ""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    blas = ""
    try:
        cfg = np.show_config(mode="dicts")
        b = cfg.get("Build Dependencies", {}).get("blas", {})
        blas = f"{b.get('name', '')} {b.get('version', '')}".strip()
    except Exception:
        pass
    threads = os.cpu_count() or 1
    try:
        from threadpoolctl import threadpool_info
        info = [i for i in threadpool_info() if i.get("user_api") == "blas"]
        if info:
            threads = max(i.get("num_threads", 1) for i in info)
            blas = blas or f"{info[0].get('internal_api', '')} {info[0].get('version', '')}".strip()
    except Exception:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model, "blas": blas, "blas_threads": int(threads)}


def cpu_baseline(s, o, reps=5, certify=None):
    """The cpu_baseline leg: the oracle (NumPy FP64, all host cores) times one PPL evaluation
    of the same (20,200,600) inputs with MP2 amplitudes, once untimed and then `reps` times
    (median reported). With `certify` = (system, amplitudes on the device) of the converged
    mixed run at (40,400,1200), the same leg also evaluates the oracle's residual
    (V + PPL(t)) / D - t of those amplitudes at sampled entries."""
    import numpy as np
    import oracle as O
    V, D = O.mp2_parts(s["L"], o, s["e_occ"], s["e_vir"])
    t = V / D
    R = O.ppl(s["L"], o, t)                  # warm-up
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        R = O.ppl(s["L"], o, t)
        times.append(time.perf_counter() - t0)
    dt = float(np.median(times))
    f = nominal(o, s["v"], s["naux"])
    assert np.isfinite(R).all()
    host = host_description()
    out = {"value": (f["build"] + f["contract"]) / dt / 1e12, "unit": "TFLOP/s", "cores": host["blas_threads"],
           "kind": "oracle", "seconds": dt, "seconds_each": [round(x, 3) for x in times], "host": host,
           "sample": f"one full oracle PPL evaluation (integrals + contraction) of the same "
                     f"({o},{s['v']},{s['naux']}) inputs with MP2 amplitudes, median of {reps} after one "
                     f"untimed run, scaled by the pair method's useful flops of one evaluation"}
    if certify is not None:
        out["c3_certification"] = oracle_residual_sampled(O, *certify)
    return out


def oracle_residual_sampled(O, s, t, reported, n_pairs=24, n_ab=40, seed=23):
    """Oracle residual of device amplitudes t at n_pairs occupied pairs x n_ab virtual pairs:
    V_ij^ab, PPL(t)_ij^ab (ppl_entry) and D from the host inputs, t[i, j] one block each.
    The full-tensor estimate sqrt(mean(d^2) o^2 v^2) is compared with the reported residual."""
    import numpy as np
    o, v, L = s["o"], s["v"], s["L"]
    Lov, Lvv = L[:, :o, o:], L[:, o:, o:]
    rng = np.random.default_rng(seed)
    d = []
    t0 = time.perf_counter()
    for _ in range(n_pairs):
        i, j = (int(x) for x in rng.integers(o, size=2))
        tij = t[i, j].cpu().numpy()
        for _ in range(n_ab):
            a, b = (int(x) for x in rng.integers(v, size=2))
            Pij = O.ppl_entry(Lvv[:, a, :], Lvv[:, b, :], tij)
            Dij = s["e_occ"][i] + s["e_occ"][j] - s["e_vir"][a] - s["e_vir"][b]
            d.append((float(Lov[:, i, a] @ Lov[:, j, b]) + Pij) / Dij - tij[a, b])
    d = np.array(d)
    est = float(np.sqrt(np.mean(d * d) * o * o * v * v))
    return {"entries": int(d.size), "max_abs": float(np.abs(d).max()), "full_tensor_estimate": est,
            "reported_residual": reported, "ratio": est / reported if reported > 0 else None,
            "seconds": round(time.perf_counter() - t0, 2)}


def measured_traffic(config):
    """HBM bytes per R+ launch from the committed hardware-counter summary, or None
    when the kernel source differs from the one measured or its R+ configuration
    (tile, split-K count) was not measured."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "contract_fp64_o20_v200_naux600_traffic.json")
    try:
        rec = json.load(open(path))
        src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    except (OSError, ValueError, KeyError):
        return None
    if hashlib.sha256(src).hexdigest()[:16] != rec.get("sha256_16"):
        return None
    return rec.get("bytes_per_launch", {}).get(f"{config[0]},{config[1]}")


def c3_leg(args):
    """Second half of the metric: wall time from inputs in HBM to an amplitude residual below
    1e-7 at (40, 400, 1200), contractive generator seed 2 (every plan resident). Plain FP64
    against BF16x3 sweeps refined in FP64, from the MP2 and from the learned start, each
    without and with DIIS (subspace 8); speed-ups like for like (both sides without, or
    both with DIIS). The same pair with DIIS also for the full linearized doubles operator
    (ladder, hole-hole ladder and ring terms), whose fixed point differs. Returns the summary and the (system, amplitudes) of the mixed + learned
    + DIIS run for the oracle's certification."""
    import numpy as np
    import torch

    import paper_2603_20912_amd as P
    from paper_2603_20912_amd import learned as Lr
    import ppl_synth

    o, v, naux, tol = 40, 400, 1200, 1e-7
    t0 = time.perf_counter()
    sysd = ppl_synth.make_system(o, v, naux, 2, "contractive")
    gen_s = time.perf_counter() - t0
    mlp = P.MLP(max_batch=1024)
    mlp.set_params(np.fromfile(args.weights, dtype="<f4"))
    # (start, precision, FP64 copy, DIIS subspace, the full linearized doubles operator: ladder,
    # hole-hole ladder and ring terms)
    runs = {"fp64": ("mp2", "fp64", False, 0, False), "bf16x3_fp64": ("mp2", "bf16x3", True, 0, False),
            "bf16x3_fp64_learned": ("learned", "bf16x3", True, 0, False),
            "fp64_diis": ("mp2", "fp64", False, 8, False), "bf16x3_fp64_diis": ("mp2", "bf16x3", True, 8, False),
            "bf16x3_fp64_learned_diis": ("learned", "bf16x3", True, 8, False),
            "fp64_diis_full_operator": ("mp2", "fp64", False, 8, True),
            "bf16x3_fp64_diis_full_operator": ("mp2", "bf16x3", True, 8, True)}
    small = ppl_synth.make_system(4, 24, 72, 99, "contractive")
    for start, prec, keep, diis, full in runs.values():   # every code path once, untimed
        Lr.time_to_tol(small, start, mlp=mlp, prec=prec, keep_fp64=keep, diis=diis, hhl=full, ring=full)
    out = {"workload": f"({o},{v},{naux}) contractive generator seed 2, amplitude residual < {tol}",
           "input_generation_s": round(gen_s, 2), "runs": {}}
    kept = None
    for label, (start, prec, keep, diis, full) in runs.items():
        torch.cuda.empty_cache()
        rep, t = Lr.time_to_tol(sysd, start, mlp=mlp, tol=tol, prec=prec, keep_fp64=keep, diis=diis, hhl=full,
                                ring=full)
        out["runs"][label] = {"seconds": round(rep["seconds"], 3), "sweeps_lp": rep["sweeps_lp"],
                              "sweeps_fp64": rep["sweeps_fp64"], "residual": rep["residual"],
                              "energy": rep["energy"], "status": rep["status"]}
        print(json.dumps({"c3": {label: out["runs"][label]}}), file=sys.stderr, flush=True)
        if label == "bf16x3_fp64_learned_diis":
            kept = (sysd, t, rep["residual"])
        else:
            del t
    mlp.close()
    r = out["runs"]
    for label in r:
        ref = "fp64_diis_full_operator" if label.endswith("full_operator") else "fp64"
        r[label]["abs_err_E_vs_fp64"] = abs(r[label]["energy"] - r[ref]["energy"])

    def ratio(a, b):
        return round(r[a]["seconds"] / r[b]["seconds"], 3)
    out["speedup"] = {"mixed_learned_vs_fp64_no_diis": ratio("fp64", "bf16x3_fp64_learned"),
                      "mixed_learned_vs_fp64_both_diis": ratio("fp64_diis", "bf16x3_fp64_learned_diis"),
                      "mixed_vs_fp64_no_diis": ratio("fp64", "bf16x3_fp64"),
                      "mixed_vs_fp64_both_diis": ratio("fp64_diis", "bf16x3_fp64_diis"),
                      "learned_vs_mp2_start_mixed_no_diis": ratio("bf16x3_fp64", "bf16x3_fp64_learned"),
                      "learned_vs_mp2_start_mixed_diis": ratio("bf16x3_fp64_diis", "bf16x3_fp64_learned_diis"),
                      "diis_vs_plain_fp64": ratio("fp64", "fp64_diis"),
                      "mixed_vs_fp64_full_operator_both_diis": ratio("fp64_diis_full_operator",
                                                                     "bf16x3_fp64_diis_full_operator")}
    return out, kept


def study_c3(args):
    """Time to an amplitude residual of 1e-7 at (40, 400, 1200), contractive generator
    seed 2: FP64, BF16x3 / BF16x6 / FP32 sweeps refined in FP64, and the same from the
    learned start, each also with DIIS (subspace 8); FP64 and BF16x3 + FP64 with DIIS for
    the iteration that also carries the hole-hole ladder, and that with the ring terms too;
    plus single-evaluation errors of
    the low-precision GEMMs."""
    import numpy as np
    import torch

    import paper_2603_20912_amd as P
    from paper_2603_20912_amd import learned as Lr
    import ppl_synth

    o, v, naux = 40, 400, 1200
    sysd = ppl_synth.make_system(o, v, naux, 2, "contractive")
    mlp = None
    if args.weights and os.path.exists(args.weights):
        mlp = P.MLP(max_batch=1024)
        mlp.set_params(np.fromfile(args.weights, dtype="<f4"))
    # warm-up of every code path on a small instance
    small = ppl_synth.make_system(4, 24, 72, 99, "contractive")
    for start, prec, keep in (("mp2", "fp64", False), ("mp2", "bf16x3", True), ("mp2", "fp32", True),
                              ("mp2", "bf16x6", True)):
        Lr.time_to_tol(small, start, mlp=mlp, prec=prec, keep_fp64=keep)
        Lr.time_to_tol(small, start, mlp=mlp, prec=prec, keep_fp64=keep, diis=8)
    Lr.time_to_tol(small, "mp2", prec="bf16x3", keep_fp64=True, diis=8, hhl=True)
    Lr.time_to_tol(small, "mp2", prec="bf16x3", keep_fp64=True, diis=8, hhl=True, ring=True)
    if mlp is not None:
        Lr.time_to_tol(small, "learned", mlp=mlp, prec="bf16x3", keep_fp64=True)
    runs = [("fp64", "mp2", "fp64", False, 0), ("bf16x3+fp64", "mp2", "bf16x3", True, 0),
            ("fp32+fp64", "mp2", "fp32", True, 0), ("bf16x6+fp64", "mp2", "bf16x6", True, 0)]
    if mlp is not None:
        runs += [("bf16x3+fp64 learned", "learned", "bf16x3", True, 0), ("fp64 learned", "learned", "fp64", False, 0)]
    # the same with DIIS (subspace of 8)
    runs += [("fp64 diis", "mp2", "fp64", False, 8), ("bf16x3+fp64 diis", "mp2", "bf16x3", True, 8),
             ("fp32+fp64 diis", "mp2", "fp32", True, 8), ("bf16x6+fp64 diis", "mp2", "bf16x6", True, 8)]
    if mlp is not None:
        runs += [("bf16x3+fp64 learned diis", "learned", "bf16x3", True, 8),
                 ("fp64 learned diis", "learned", "fp64", False, 8)]
    runs = [r + (False, False) for r in runs]
    # the linearized doubles iteration with the hole-hole ladder too, then also with the
    # ring terms (each its own fixed point, compared with its own FP64 run)
    runs += [("fp64 diis hhl", "mp2", "fp64", False, 8, True, False),
             ("bf16x3+fp64 diis hhl", "mp2", "bf16x3", True, 8, True, False),
             ("fp64 diis hhl ring", "mp2", "fp64", False, 8, True, True),
             ("bf16x3+fp64 diis hhl ring", "mp2", "bf16x3", True, 8, True, True)]
    out = {"config": {"o": o, "v": v, "naux": naux, "generator": "contractive", "seed": 2, "tol": 1e-7}}
    refs = {}
    for label, start, prec, keep, diis, hhl, ring in runs:
        torch.cuda.empty_cache()
        free_gib = torch.cuda.mem_get_info()[0] / 2 ** 30
        rep, t = Lr.time_to_tol(sysd, start, mlp=mlp, tol=1e-7, prec=prec, keep_fp64=keep, diis=diis, hhl=hhl,
                                ring=ring)
        row = {"seconds": round(rep["seconds"], 3), "sweeps_lp": rep["sweeps_lp"], "sweeps_fp64": rep["sweeps_fp64"],
               "residual": rep["residual"], "energy": rep["energy"], "status": rep["status"],
               "resident": rep["resident"], "free_GiB_before": round(free_gib, 1), "kernel_ms": rep["kernel_ms"]}
        if (hhl, ring) not in refs:
            refs[(hhl, ring)] = (t.clone(), rep["energy"])
        else:
            ref_t, ref_E = refs[(hhl, ring)]
            row["rel_err_t_vs_fp64"] = (torch.linalg.norm(t - ref_t) / torch.linalg.norm(ref_t)).item()
            row["abs_err_E_vs_fp64"] = abs(rep["energy"] - ref_E)
        out[label] = row
        print(json.dumps({label: row}), file=sys.stderr, flush=True)
        del t
        torch.cuda.empty_cache()
    # single-evaluation errors of R (MP2 amplitudes) against the FP64 path
    d = Lr.upload_system(sysd)
    Rs = {}
    for prec in ("fp64", "fp32", "bf16x3", "bf16x6"):
        eng = P.PPL(o, v, naux, prec=prec)
        tm, _ = eng.mp2(d["L"], d["e_occ"], d["e_vir"])
        eng.build(d["L"])
        Rs[prec] = eng.contract(tm)
        eng.close()
        del eng
        torch.cuda.empty_cache()
    for prec in ("fp32", "bf16x3", "bf16x6"):
        out[f"single_R_rel_err_{prec}"] = (torch.linalg.norm(Rs[prec] - Rs["fp64"]) /
                                           torch.linalg.norm(Rs["fp64"])).item()
    print(json.dumps({"study": out}), flush=True)


def study_batched(args):
    """The 32 uneven instances of the batched configuration (o in [8, 24], v in [80, 240],
    naux = 3v): contraction of all instances by one grouped persistent launch replayed
    from a hipGraph, against one autotuned plan per instance launched one after another;
    and the whole evaluation from L (integral builds as concurrent branches, then the
    grouped contraction) in one graph, against the plans' builds and contractions in turn
    (the sequential builds include their symmetry check of L, a host round trip each)."""
    import torch

    import paper_2603_20912_amd as P
    import ppl_synth

    shapes = ppl_synth.batched_shapes(32, seed=4)
    tup = [(d["o"], d["v"], d["naux"]) for d in shapes]
    flops = sum(nominal(*t)["contract"] for t in tup)
    out = {"instances": len(tup), "shapes": tup, "useful_contract_flops": flops}
    stream = torch.cuda.Stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    with torch.cuda.stream(stream):
        bflops = sum(nominal(*t)["build"] for t in tup)
        out["useful_build_flops"] = bflops
        for prec in ("fp64", "fp32"):
            seq_ms = seq_full_ms = 0.0
            for d, (o, v, naux) in zip(shapes, tup):
                sysd = ppl_synth.make_system(o, v, naux, d["seed"])
                L = torch.from_numpy(sysd["L"]).cuda()
                t = torch.from_numpy(ppl_synth.make_amplitudes(o, v, d["seed"] + 5000)).cuda()
                eng = P.PPL(o, v, naux, prec=prec, stream=stream)
                eng.build(L)
                R = eng.contract(t)              # the tuner then times these operands
                eng.autotune(reps=3)
                e0.record(stream)
                for _ in range(reps):
                    eng.contract(t, R)
                e1.record(stream)
                e1.synchronize()
                seq_ms += e0.elapsed_time(e1) / reps
                # the same plan's whole evaluation from L (build, then contraction)
                e0.record(stream)
                for _ in range(3):
                    eng.build(L)
                    eng.contract(t, R)
                e1.record(stream)
                e1.synchronize()
                seq_full_ms += e0.elapsed_time(e1) / 3
                eng.close()
                del L, t, R, eng
            torch.cuda.empty_cache()
            b = P.Batch(tup, prec=prec, stream=stream)
            Ls, ts = [], []
            for d, (o, v, naux) in zip(shapes, tup):
                Ls.append(torch.from_numpy(ppl_synth.make_system(o, v, naux, d["seed"])["L"]).cuda())
                ts.append(torch.from_numpy(ppl_synth.make_amplitudes(o, v, d["seed"] + 5000)).cuda())
            Rs = [torch.empty_like(t) for t in ts]
            stream.synchronize()
            t0 = time.perf_counter()
            b.build(Ls)
            stream.synchronize()
            build_s = time.perf_counter() - t0
            b.contract(ts, Rs)
            e0.record(stream)
            for _ in range(reps):
                b.contract(ts, Rs)
            e1.record(stream)
            e1.synchronize()
            model_ms = e0.elapsed_time(e1) / reps
            b.autotune(reps=2)
            b.contract(ts, Rs)
            e0.record(stream)
            for _ in range(reps):
                b.contract(ts, Rs)
            e1.record(stream)
            e1.synchronize()
            eager_ms = e0.elapsed_time(e1) / reps
            b.capture(ts, Rs)
            b.replay()
            e0.record(stream)
            for _ in range(reps):
                b.replay()
            e1.record(stream)
            e1.synchronize()
            graph_ms = e0.elapsed_time(e1) / reps
            # the whole evaluation from L and t2 (builds + contraction) in one graph
            b.capture(ts, Rs, Ls=Ls)
            b.replay()
            e0.record(stream)
            for _ in range(3):
                b.replay()
            e1.record(stream)
            e1.synchronize()
            graph_full_ms = e0.elapsed_time(e1) / 3
            out[prec] = {"graph_ms": round(graph_ms, 3), "eager_grouped_ms": round(eager_ms, 3),
                         "eager_grouped_model_tiles_ms": round(model_ms, 3),
                         "sequential_ms": round(seq_ms, 3), "graph_tflops": round(flops / graph_ms / 1e9, 2),
                         "sequential_tflops": round(flops / seq_ms / 1e9, 2),
                         "speedup_vs_sequential": round(seq_ms / graph_ms, 3), "build_s": round(build_s, 3),
                         "graph_build_and_contract_ms": round(graph_full_ms, 3),
                         "sequential_build_and_contract_ms": round(seq_full_ms, 3),
                         "speedup_build_and_contract_vs_sequential": round(seq_full_ms / graph_full_ms, 3),
                         "build_and_contract_tflops": round((flops + bflops) / graph_full_ms / 1e9, 2)}
            print(json.dumps({prec: out[prec]}), file=sys.stderr, flush=True)
            b.close()
            del b, Ls, ts, Rs
            torch.cuda.empty_cache()
    print(json.dumps({"study": out}), flush=True)


# C-split times (s) of the paper's contraction benchmark (Tab. xc-split) for the shapes
# with nvec = 5N whose t, R and L fit one MI355X next to a streaming workspace
PAPER_C_SPLIT = {(100, 700, 4000): {"CuPy GH200": 306.6, "PyTorch GH200": 355.9, "CuPy H100": 461.5,
                                    "PyTorch H100": 330.5},
                 (100, 800, 4500): {"CuPy GH200": 495.0, "PyTorch GH200": 587.1, "CuPy H100": 809.7,
                                    "PyTorch H100": 496.2},
                 (50, 950, 10000): {"CuPy GH200": 763.0, "PyTorch GH200": 574.6, "CuPy H100": 1006.4,
                                    "PyTorch H100": 673.0}}


def study_paper(args):
    """One FP64 PPL evaluation at a shape of the paper's contraction benchmark
    (Tab. xc-split: N = 800, nocc = 100, nvec = 5N = 4000, nvir = 700 by default; with
    --paper-shape 100,800,4500 the N = 900 one, with 50,950,10000 the N = 1000 one with
    nocc = 50 and nvec = 10N), on one GPU.

    V+- would take about 960 GB, so the plan streams: each row batch is built from the
    Cholesky vectors and contracted at once, with t, R and L resident in HBM. Inputs are
    drawn on the device (same recipe as the small configurations, contractive amplitude).
    Timed: whole ppl_contract calls (staging, every batch's build and contraction,
    packing and unpacking), after one untimed call."""
    import torch

    import paper_2603_20912_amd as P
    import ppl_synth

    o, v, naux = (int(x) for x in args.paper_shape.split(","))
    dense = {"build": 2.0 * naux * v ** 4, "contract": 2.0 * o * o * v ** 4}
    paper = PAPER_C_SPLIT.get((o, v, naux), {})
    out = {"shape": {"N": o + v, "nocc": o, "nvir": v, "nvec": naux}, "precision": "fp64",
           "dense_flops": dense["build"] + dense["contract"], "paper_seconds_C_split": paper}
    t0 = time.perf_counter()
    sysd = ppl_synth.make_system_device(o, v, naux, 21)
    t = ppl_synth.make_amplitudes_device(o, v, 22)
    R = torch.empty_like(t)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    print(json.dumps({"inputs_s": round(time.perf_counter() - t0, 2),
                      "free_GB": torch.cuda.mem_get_info()[0] / 1e9}), file=sys.stderr, flush=True)
    eng = P.PPL(o, v, naux, prec="fp64", build_scratch=64 << 30, contract_only=True)
    if args.contract_config:
        eng.set_contract_config(*[int(x) for x in args.contract_config.split(",")])
    info = eng.info
    # useful flops as the plan executes them (upper-triangle build steps over packed columns)
    out["useful_flops"] = info["flops_build"] + info["flops_contract"]
    out["useful_flops_build"] = info["flops_build"]
    out["plan"] = {k: info[k] for k in ("resident", "n_batches", "max_step_pairs", "workspace_bytes",
                                        "tile_build", "tile_contract", "splits_contract",
                                        "tile_contract_minus", "splits_contract_minus")}
    print(json.dumps({"plan": out["plan"]}), file=sys.stderr, flush=True)
    eng.build(sysd["L"])
    times = []
    for k in range(1 + args.steps):
        if k == 1:
            eng.profile(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        eng.contract(t, R)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        print(json.dumps({"evaluation": k, "seconds": round(times[-1], 3), "timed": k > 0}),
              file=sys.stderr, flush=True)
    prof = eng.profile_read()
    eng.profile(False)
    eng.close()
    del eng
    torch.cuda.empty_cache()
    sec = sum(times[1:]) / len(times[1:])
    # pair symmetry R_ij^ab = R_ji^ba, one occupied row at a time (R is 39 GB)
    num = den = 0.0
    for i in range(o):
        d = R[i] - R[:, i].transpose(1, 2)
        num += (d * d).sum().item()
        den += (R[i] * R[i]).sum().item()
    sym = (num / den) ** 0.5
    out.update({"seconds": round(sec, 3), "seconds_each": [round(x, 3) for x in times[1:]],
                "untimed_first_s": round(times[0], 3),
                "useful_tflops": round(out["useful_flops"] / sec / 1e12, 2),
                "pct_fp64_mfma_peak": round(100.0 * out["useful_flops"] / sec / 1e12 / PEAK_FP64_TFLOPS, 2),
                "dense_equivalent_tflops": round(out["dense_flops"] / sec / 1e12, 2),
                "speedup_vs_best_paper_time": round(min(paper.values()) / sec, 2) if paper else None,
                "pair_symmetry_rel": sym, "finite": all(torch.isfinite(R[i]).all().item() for i in range(o))})
    n = args.steps
    out["kernels"] = {k: {"launches": d["launches"] // n, "s": round(d["ms"] / n / 1e3, 3),
                          "tflops": round(d["flops"] / (d["ms"] * 1e-3) / 1e12, 2) if d["ms"] > 0 and d["flops"] > 0
                          else None} for k, d in prof.items() if d["launches"]}
    print(json.dumps({"study": out}), flush=True)


def study_terms(args):
    """Times of the CCSD terms next to the ladder at (40, 400, 1200), FP64, inputs in HBM:
    the ladder PPL(t2), the ladder with singles PPL(t2 + t1 t1), the hole-hole ladder
    sum_kl (ki|lj) t_kl^ab and the ring terms (integrals from L included in both), each
    averaged over 5 calls."""
    import numpy as np
    import torch

    import paper_2603_20912_amd as P
    import ppl_synth

    o, v, naux = 40, 400, 1200
    sysd = ppl_synth.make_system(o, v, naux, 2, "contractive")
    L = torch.from_numpy(sysd["L"]).cuda()
    t2 = torch.from_numpy(ppl_synth.make_amplitudes(o, v, 3)).cuda()
    t1 = torch.from_numpy(0.05 * np.random.default_rng(19).standard_normal((o, v))).cuda()
    R = torch.empty_like(t2)
    eng = P.PPL(o, v, naux)
    eng.build(L)
    Pp, Pm, Np, Nm = v * (v + 1) // 2, v * (v - 1) // 2, o * (o + 1) // 2, o * (o - 1) // 2
    ring_scratch = torch.empty(P.ppl_ring_scratch_bytes(o, v, naux), dtype=torch.uint8, device="cuda")
    calls = {"ppl": lambda: eng.contract(t2, R), "ppl_tau": lambda: eng.contract(t2, R, t1=t1),
             "hhl": lambda: eng.hhl(L, t2, R), "ring": lambda: P.ring(L, t2, R, scratch=ring_scratch)}
    ov = o * v
    flops = {"ppl": nominal(o, v, naux)["contract"], "ppl_tau": nominal(o, v, naux)["contract"],
             "hhl": 2.0 * (Pp * Np * Np + Pm * Nm * Nm),
             # three (ov)^3 GEMMs and the (kc|jb), (kj|bc) integrals
             "ring": 6.0 * ov ** 3 + 4.0 * ov * ov * naux}
    out = {"config": {"o": o, "v": v, "naux": naux, "precision": "fp64"}}
    for name, fn in calls.items():
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            fn()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / 5
        out[name] = {"ms": round(ms, 3), "useful_tflops": round(flops[name] / ms / 1e9, 2)}
    eng.close()
    print(json.dumps({"study": out}), flush=True)


def study_kernels(args):
    """Every MFMA kernel family once more after an untimed first call, for per-kernel profiles
    (rocprofv3 kernel traces and counters): at (40, 400, 1200), contractive generator seed 2
    with N(0,1) pair-symmetric amplitudes, the integral build and one contraction in FP32,
    BF16x3 and BF16x6 (contract-only plans, the planner's tiles), the hole-hole ladder and
    the ring terms in FP64; the learned-start inference (BF16 MFMA) at (30, 300, 900); the
    32 uneven batched instances (the grouped persistent contraction) in FP64 and FP32."""
    import numpy as np
    import torch

    import paper_2603_20912_amd as P
    import ppl_synth

    # one plain 1 GiB device copy first: the reference that calibrates byte counters
    x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    del x, y
    o, v, naux = 40, 400, 1200
    sysd = ppl_synth.make_system(o, v, naux, 2, "contractive")
    L = torch.from_numpy(sysd["L"]).cuda()
    t = torch.from_numpy(ppl_synth.make_amplitudes(o, v, 3)).cuda()
    R = torch.empty_like(t)
    out = {}
    for prec in ("fp32", "bf16x3", "bf16x6"):
        eng = P.PPL(o, v, naux, prec=prec, contract_only=True)
        for _ in range(2):
            eng.build(L)
            eng.contract(t, R)
        torch.cuda.synchronize()
        out[prec] = {"contract_config": list(eng.contract_config())}
        eng.close()
        del eng
        torch.cuda.empty_cache()
        print(json.dumps({"done": prec}), file=sys.stderr, flush=True)
    eng = P.PPL(o, v, naux, prec="fp64", contract_only=True)
    for _ in range(2):
        eng.hhl(L, t, R)
    eng.close()
    del eng
    torch.cuda.empty_cache()
    scratch = torch.empty(P.ppl_ring_scratch_bytes(o, v, naux), dtype=torch.uint8, device="cuda")
    for _ in range(2):
        P.ring(L, t, R, scratch=scratch)
    torch.cuda.synchronize()
    del scratch, L, t, R
    torch.cuda.empty_cache()
    print(json.dumps({"done": "hhl, ring"}), file=sys.stderr, flush=True)
    # learned-start inference on a held-out instance
    o5, v5, n5 = 30, 300, 900
    s5 = ppl_synth.make_system(o5, v5, n5, 3000, "contractive")
    d = {k: torch.from_numpy(np.ascontiguousarray(s5[k])).cuda() for k in ("L", "e_occ", "e_vir")}
    eng = P.PPL(o5, v5, n5, contract_only=False)
    tm, _ = eng.mp2(d["L"], d["e_occ"], d["e_vir"])
    mlp = P.MLP(max_batch=1024)
    mlp.set_params(np.fromfile(args.weights, dtype="<f4"))
    for _ in range(2):
        g = mlp.guess(eng, tm, d["e_occ"], d["e_vir"])
    torch.cuda.synchronize()
    mlp.close()
    eng.close()
    del eng, tm, g, d
    torch.cuda.empty_cache()
    print(json.dumps({"done": "mlp"}), file=sys.stderr, flush=True)
    # the batched instances
    shapes = ppl_synth.batched_shapes(32, seed=4)
    tup = [(x["o"], x["v"], x["naux"]) for x in shapes]
    Ls = [torch.from_numpy(ppl_synth.make_system(*sh, x["seed"])["L"]).cuda() for sh, x in zip(tup, shapes)]
    ts = [torch.from_numpy(ppl_synth.make_amplitudes(sh[0], sh[1], x["seed"] + 5000)).cuda()
          for sh, x in zip(tup, shapes)]
    Rs = [torch.empty_like(x) for x in ts]
    for prec in ("fp64", "fp32"):
        b = P.Batch(tup, prec=prec)
        b.build(Ls)
        for _ in range(2):
            b.contract(ts, Rs)
        torch.cuda.synchronize()
        b.close()
        del b
        torch.cuda.empty_cache()
        print(json.dumps({"done": f"batched {prec}"}), file=sys.stderr, flush=True)
    print(json.dumps({"study": out}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c3", action="store_true",
                    help="skip the time-to-residual leg at (40, 400, 1200) (the metric's second half)")
    ap.add_argument("--contract-config", default="",
                    help="tile_plus,splits_plus,tile_minus,splits_minus instead of autotuning")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run one plain 1 GiB device copy (reference for hardware byte counters)")
    ap.add_argument("--study", default="", help="c3: time-to-1e-7 study at (40, 400, 1200); "
                    "batched: the 32 uneven instances, grouped graph launch vs one plan each; "
                    "paper: one streamed FP64 evaluation at (nocc, nvir, nvec) = (100, 700, 4000); "
                    "terms: ladder, ladder with singles and hole-hole ladder at (40, 400, 1200); "
                    "kernels: every MFMA kernel family once, for rocprofv3 profiles")
    ap.add_argument("--paper-shape", default="100,700,4000", help="nocc,nvir,nvec of --study paper")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_2603_20912_amd", "weights", "mlp_start.f32"))
    args = ap.parse_args()
    if args.study == "c3":
        return study_c3(args)
    if args.study == "batched":
        return study_batched(args)
    if args.study == "paper":
        return study_paper(args)
    if args.study == "terms":
        return study_terms(args)
    if args.study == "kernels":
        return study_kernels(args)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(every box has a single MI355X); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2603_20912_amd as P
    import ppl_synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    s = ppl_synth.make_system(O_, V_, NAUX_, SEED_, "literal")
    L = torch.from_numpy(s["L"]).to(dev)
    eo = torch.from_numpy(s["e_occ"]).to(dev)
    ev = torch.from_numpy(s["e_vir"]).to(dev)
    t = torch.zeros((O_, O_, V_, V_), dtype=torch.float64, device=dev)
    R = torch.empty_like(t)
    eng = P.PPL(O_, V_, NAUX_, prec="fp64")
    f = nominal(O_, V_, NAUX_)
    assert f["build"] == eng.info["flops_build"] and f["contract"] == eng.info["flops_contract"]
    flops_step = f["build"] + (SWEEPS + 1) * f["contract"]

    def step():
        eng.iterate(L, eo, ev, t, max_sweeps=SWEEPS, tol=0.0, diverge_factor=0.0, history=False)
        eng.contract(t, R)

    if args.copy_calibration:
        x = torch.ones(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB read, 1 GiB written
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y

    # one-time setup outside the timed region: build V+- once and let the
    # library's autotuner pick the contraction tiles and split-K counts
    eng.build(L)
    if args.contract_config:
        eng.set_contract_config(*[int(x) for x in args.contract_config.split(",")])
    else:
        # the tuner times the operands in the workspace, and the MFMA rate depends on
        # their values through the power draw: tune on the workload's own amplitudes
        step()
        eng.autotune(reps=3)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    eng.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = eng.profile_read()
    eng.profile(False)
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = flops_step / (ms_step * 1e-3) / 1e12
    assert torch.isfinite(R).all().item()

    cp = prof["contract_plus"]
    avg_ms = cp["ms"] / max(cp["launches"], 1)
    fl_launch = cp["flops"] / max(cp["launches"], 1)
    achieved = fl_launch / (avg_ms * 1e-3) / 1e12
    kernels = {k: {"launches": d["launches"], "avg_ms": d["ms"] / d["launches"] if d["launches"] else 0.0,
                   "tflops": (d["flops"] / (d["ms"] * 1e-3) / 1e12) if d["ms"] > 0 and d["flops"] > 0 else None}
               for k, d in prof.items()}
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "PPL FP64 (o=20, v=200, naux=600), literal generator seed 1: "
                               "V+- build + MP2 start + 10 Jacobi sweeps + 1 evaluation",
                   "o": O_, "v": V_, "naux": NAUX_, "sweeps": SWEEPS, "precision": "fp64",
                   "useful_flops_per_step": flops_step,
                   "pct_fp64_mfma_peak": round(100.0 * value / PEAK_FP64_TFLOPS, 2),
                   "contract_config": list(eng.contract_config())},
        "roofline": {"bound": "mfma", "kernel": "R+ contraction GEMM (FP64 MFMA 16x16x4)",
                     "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
                     "traffic": measured_traffic(eng.contract_config()),
                     "flops_per_launch": fl_launch, "avg_launch_ms": round(avg_ms, 4)},
        "kernels": kernels,
    }
    eng.close()
    del eng, L, eo, ev, t, R
    torch.cuda.empty_cache()
    kept = None
    if not args.no_c3:
        out["time_to_residual"], kept = c3_leg(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(s, O_, certify=kept)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
