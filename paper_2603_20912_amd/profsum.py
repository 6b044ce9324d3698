"""Summaries of rocprofv3 runs of bench.py for the profiles/ folder.

    python -m paper_2603_20912_amd.profsum --trace-stats TRACE_kernel_stats.csv \
        --counters 0,4,8,6 FETCH_counter_collection.csv WRITE_counter_collection.csv [--counters ...] \
        --command "rocprofv3 ..." [--command ...] --md OUT.md --json OUT.json

Inputs are the CSV files of one `--kernel-trace --stats` run and, per contraction
configuration, one FETCH_SIZE and one WRITE_SIZE counter run of
`bench.py --steps 1 --warmup 0 --contract-config CFG --copy-calibration`.

Calibration: the counter runs begin with one plain 1 GiB device-to-device copy.
The copy dispatch whose WRITE_SIZE is closest to 1 GiB scales both counters
(bytes moved / counter reading), so the traffic of the other kernels is stated
in bytes.

The R+ contraction launches are the GEMM dispatches whose grid matches the R+
grid of the configuration (tile shape from ppl_tile_dims, split-K count after the
library's clamping); each is counted together with the split-K reduction that
follows it, which is what the bench times as one R+ launch. The JSON gives the
bytes per R+ launch keyed by "tile,splits", with the sha256 of the GEMM source,
so that the bench reports traffic only for the kernel code that was measured.

    python -m paper_2603_20912_amd.profsum mfma --counters MFMA_counter_collection.csv \
        --command "rocprofv3 ..." --md OUT.md

summarises one `--pmc SQ_INSTS_VALU_MFMA_MOPS_F64 GRBM_GUI_ACTIVE` run: per
kernel, the FP64 matrix-core work it executed (the counter counts units of 512
flops, padded tile rows included) over its profiled dispatch time, as TF/s and
as a fraction of the FP64 MFMA peak, and the shader clock (GRBM_GUI_ACTIVE is
summed over the 8 XCDs).
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GEMM_SRC = "paper_2603_20912_amd/csrc/gemm.hip"
GIB_KIB = 1024.0 * 1024.0


def pairs_plus(n):
    return n * (n + 1) // 2


def pad64(k):
    return (k + 63) // 64 * 64


def short_name(k):
    k = k.replace("void ", "").replace("ppl::", "")
    return k.split("(")[0] if "<" not in k else k[: k.index(">") + 1]


def rplus_grid(tile, splits, o, v, kc=16):
    """Threads of the R+ GEMM launch of (tile, splits) (split-K configurations only)."""
    from . import ppl_tile_dims
    bm, bn, th = ppl_tile_dims(tile)
    M, N, K = pairs_plus(o), pairs_plus(v), pad64(pairs_plus(v))
    nk = K // kc
    s = max(1, min(splits, nk))
    kps = (nk + s - 1) // s
    s = (nk + kps - 1) // kps
    return -(-M // bm) * -(-N // bn) * s * th


def read_counters(path):
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    return rows


def calibration_dispatch(write_rows):
    """Dispatch id of the 1 GiB calibration copy: the copy whose WRITE_SIZE is closest to 1 GiB."""
    copies = [r for r in write_rows if "copy" in r["Kernel_Name"].lower()]
    best = min(copies, key=lambda r: abs(float(r["Counter_Value"]) - GIB_KIB))
    if abs(float(best["Counter_Value"]) - GIB_KIB) > 0.02 * GIB_KIB:
        raise SystemExit("no 1 GiB calibration copy in the WRITE_SIZE run (bench.py --copy-calibration)")
    return int(best["Dispatch_Id"])


def per_launch(fetch_rows, write_rows, fscale, wscale, grid):
    """Scaled bytes of each R+ GEMM dispatch plus the reduction dispatch right after it."""
    w = {int(r["Dispatch_Id"]): r for r in write_rows}
    out = []
    for i, r in enumerate(fetch_rows):
        if "gemm_nt_kernel<double" not in r["Kernel_Name"] or "MapGrid" not in r["Kernel_Name"]:
            continue
        if int(r["Grid_Size"]) != grid:
            continue
        ids = [int(r["Dispatch_Id"])]
        if i + 1 < len(fetch_rows) and "splitk_reduce" in fetch_rows[i + 1]["Kernel_Name"]:
            ids.append(int(fetch_rows[i + 1]["Dispatch_Id"]))
        fb = sum(float(next(x for x in fetch_rows if int(x["Dispatch_Id"]) == d)["Counter_Value"]) for d in ids)
        wb = sum(float(w[d]["Counter_Value"]) for d in ids)
        out.append((fb * fscale + wb * wscale) * 1024.0)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--trace-stats", required=True)
    ap.add_argument("--counters", nargs=3, action="append", metavar=("CFG", "FETCH_CSV", "WRITE_CSV"), default=[])
    ap.add_argument("--command", action="append", default=[])
    ap.add_argument("--o", type=int, default=20)
    ap.add_argument("--v", type=int, default=200)
    ap.add_argument("--naux", type=int, default=600)
    ap.add_argument("--md", required=True)
    ap.add_argument("--json", required=True)
    a = ap.parse_args(argv)

    sha = hashlib.sha256(open(os.path.join(ROOT, GEMM_SRC), "rb").read()).hexdigest()[:16]
    stats = list(csv.DictReader(open(a.trace_stats)))
    stats.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"# FP64 contraction and build kernels, PPL step at (o, v, naux) = ({a.o}, {a.v}, {a.naux})", "",
             "Commands (run from the repository root on one MI355X, ROCm 7.2, `export TMPDIR=/tmp`):", "", "```"]
    lines += a.command + ["```", "",
                          f"Kernel source: `{GEMM_SRC}` sha256[:16] = `{sha}`.", "",
                          "## Kernel trace summary (`--kernel-trace --stats`)", "",
                          "| calls | avg ms | % time | kernel |", "|---:|---:|---:|---|"]
    for r in stats[:12]:
        lines.append(f"| {r['Calls']} | {float(r['AverageNs']) / 1e6:.4f} | {float(r['Percentage']):.2f} | "
                     f"`{short_name(r['Name'])}` |")
    rec = {"kernel": "R+ contraction GEMM with its split-K reduction", "source": GEMM_SRC, "sha256_16": sha,
           "workload": f"fp64 ({a.o},{a.v},{a.naux})", "bytes_per_launch": {}, "calibration": {}}
    algo = {}
    M, N, K = pairs_plus(a.o), pairs_plus(a.v), pad64(pairs_plus(a.v))
    for cfg, fpath, wpath in a.counters:
        c = [int(x) for x in cfg.split(",")]
        fr, wr = read_counters(fpath), read_counters(wpath)
        cal = calibration_dispatch(wr)
        fc = next(r for r in fr if int(r["Dispatch_Id"]) == cal)
        wc = next(r for r in wr if int(r["Dispatch_Id"]) == cal)
        if fc["Kernel_Name"] != wc["Kernel_Name"]:
            raise SystemExit("the FETCH_SIZE and WRITE_SIZE runs dispatched different kernels")
        fscale = GIB_KIB / float(fc["Counter_Value"])   # the copy read 1 GiB
        wscale = GIB_KIB / float(wc["Counter_Value"])   # and wrote 1 GiB
        launches = per_launch(fr, wr, fscale, wscale, rplus_grid(c[0], c[1], a.o, a.v))
        if not launches:
            raise SystemExit(f"no R+ launch of config {cfg} found in {fpath}")
        key = f"{c[0]},{c[1]}"
        rec["bytes_per_launch"][key] = sum(launches) / len(launches)
        rec["calibration"][key] = {"fetch_scale": fscale, "write_scale": wscale}
        s_eff = rplus_grid(c[0], c[1], a.o, a.v) // rplus_grid(c[0], 1, a.o, a.v)
        # V+ and S' read once, R+ written once, split-K slices written once and read once
        algo[key] = 8.0 * (N * K + M * K + M * K + (2 * s_eff * M * K if s_eff > 1 else 0))
        # per-kernel table for this configuration
        kf, kw, kn = defaultdict(float), defaultdict(float), defaultdict(int)
        wmap = {int(r["Dispatch_Id"]): r for r in wr}
        for r in fr:
            d = int(r["Dispatch_Id"])
            if d not in wmap:
                continue
            k = short_name(r["Kernel_Name"])
            kf[k] += float(r["Counter_Value"]) * fscale
            kw[k] += float(wmap[d]["Counter_Value"]) * wscale
            kn[k] += 1
        lines += ["", f"## Hardware byte counters, contraction config {cfg} (KiB per dispatch, calibrated)", "",
                  f"Calibration: FETCH_SIZE x {fscale:.4f}, WRITE_SIZE x {wscale:.4f} (one 1 GiB device copy).", "",
                  "| kernel | dispatches | FETCH KiB | WRITE KiB | GB / dispatch |", "|---|---:|---:|---:|---:|"]
        for k in sorted(kf, key=lambda k: -(kf[k] + kw[k]) / kn[k])[:10]:
            lines.append(f"| `{k}` | {kn[k]} | {kf[k] / kn[k]:.0f} | {kw[k] / kn[k]:.0f} | "
                         f"{(kf[k] + kw[k]) / kn[k] * 1024 / 1e9:.3f} |")
        lines += ["", f"R+ launch (GEMM + reduction) of config {cfg}: {rec['bytes_per_launch'][key] / 1e9:.3f} GB "
                  f"measured over {len(launches)} launches; algorithmic {algo[key] / 1e9:.3f} GB "
                  f"(V+ {N} x {K}, S' {M} x {K}, the split-K slices written and read once, R+ {M} x {K}, 8 B each)."]
    os.makedirs(os.path.dirname(os.path.abspath(a.md)), exist_ok=True)
    open(a.md, "w").write("\n".join(lines) + "\n")
    json.dump(rec, open(a.json, "w"), indent=1)
    print(f"wrote {a.md} and {a.json}")


FP64_MFMA_PEAK_TFS = 78.6


def mfma_main(argv):
    ap = argparse.ArgumentParser(description="per-kernel FP64 MFMA work from one rocprofv3 --pmc run")
    ap.add_argument("--counters", required=True)
    ap.add_argument("--command", action="append", default=[])
    ap.add_argument("--md", required=True)
    a = ap.parse_args(argv)
    mops, gui, span, name = defaultdict(float), defaultdict(float), {}, {}
    for r in csv.DictReader(open(a.counters)):
        d = int(r["Dispatch_Id"])
        name[d] = short_name(r["Kernel_Name"])
        span[d] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
        if r["Counter_Name"] == "SQ_INSTS_VALU_MFMA_MOPS_F64":
            mops[d] += float(r["Counter_Value"])
        elif r["Counter_Name"] == "GRBM_GUI_ACTIVE":
            gui[d] += float(r["Counter_Value"])
    per = defaultdict(lambda: [0, 0.0, 0.0, 0.0])
    for d, k in name.items():
        p = per[k]
        p[0] += 1
        p[1] += span[d]
        p[2] += mops[d] * 512.0
        p[3] += gui[d] / 8.0
    sha = hashlib.sha256(open(os.path.join(ROOT, GEMM_SRC), "rb").read()).hexdigest()[:16]
    lines = ["# FP64 MFMA work per kernel, PPL step at (o, v, naux) = (20, 200, 600)", "",
             "Commands (run from the repository root on one MI355X, ROCm 7.2, `export TMPDIR=/tmp`):", "", "```"]
    lines += a.command + ["```", "", f"Kernel source: `{GEMM_SRC}` sha256[:16] = `{sha}`.", "",
                          "TF/s = SQ_INSTS_VALU_MFMA_MOPS_F64 x 512 flops over the profiled dispatch time "
                          f"(padded tile rows included); peak {FP64_MFMA_PEAK_TFS} TF/s. Clock from "
                          "GRBM_GUI_ACTIVE / 8 XCDs, shown for dispatches of 0.5 ms or more (launch overhead "
                          "inflates it on short ones).", "",
                          "| kernel | dispatches | avg ms | MFMA F64 TF/s | % of peak | clock GHz |",
                          "|---|---:|---:|---:|---:|---:|"]
    for k, (n, t, fl, cyc) in sorted(per.items(), key=lambda kv: -kv[1][1])[:14]:
        if t <= 0:
            continue
        tf = fl / t / 1e12
        clk = f"{cyc / t / 1e9:.2f}" if t / n >= 5e-4 else "-"
        lines.append(f"| `{k}` | {n} | {t / n * 1e3:.4f} | {tf:.2f} | {100 * tf / FP64_MFMA_PEAK_TFS:.1f} | {clk} |")
    os.makedirs(os.path.dirname(os.path.abspath(a.md)), exist_ok=True)
    open(a.md, "w").write("\n".join(lines) + "\n")
    print(f"wrote {a.md}")


PEAK_TFS = {"F64": 78.6, "F32": 157.3, "BF16": 2500.0}   # MI355X dense matrix peaks
# flops per unit of SQ_INSTS_VALU_MFMA_MOPS_<type> (checked against the known work of the
# FP64 ring GEMM, the FP32 contraction and the BF16x3 contraction, padded rows included)
MOPS_FLOPS = {"F64": 512.0, "F32": 512.0, "BF16": 512.0}
N_SIMD = 1024                                               # 256 CUs x 4 SIMDs


def _per_dispatch(path):
    """{dispatch id: {"name", "grid", "t" (s), counter: value}} of one counter CSV."""
    out = {}
    for r in csv.DictReader(open(path)):
        d = int(r["Dispatch_Id"])
        e = out.setdefault(d, {"name": short_name(r["Kernel_Name"]), "grid": int(r["Grid_Size"]),
                               "t": (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9})
        e[r["Counter_Name"]] = e.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return out


def kernels_main(argv):
    """Per-kernel summary of one --kernel-trace run and --pmc runs of the same command:
    time, executed matrix-core work by type against its peak, matrix-core busy fraction,
    clock, LDS bank conflicts and LDS-issue waits, and calibrated HBM bytes."""
    ap = argparse.ArgumentParser(description=kernels_main.__doc__)
    ap.add_argument("--trace", required=True, help="kernel_trace.csv of the --kernel-trace run")
    ap.add_argument("--mfma", required=True, help="counter CSV with SQ_INSTS_VALU_MFMA_MOPS_*, "
                    "SQ_VALU_MFMA_BUSY_CYCLES and GRBM_GUI_ACTIVE")
    ap.add_argument("--lds", required=True, help="counter CSV with SQ_LDS_BANK_CONFLICT, SQ_INSTS_LDS, "
                    "SQ_WAIT_INST_LDS and SQ_WAVE_CYCLES")
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--command", action="append", default=[])
    ap.add_argument("--title", required=True)
    ap.add_argument("--md", required=True)
    ap.add_argument("--top", type=int, default=30)
    a = ap.parse_args(argv)
    tr = defaultdict(lambda: [0, 0.0])       # (kernel, grid) -> dispatches, seconds
    for r in csv.DictReader(open(a.trace)):
        grid = int(r["Grid_Size"]) if "Grid_Size" in r else \
            int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
        k = (short_name(r["Kernel_Name"]), grid)
        tr[k][0] += 1
        tr[k][1] += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9

    def group(path):
        g = defaultdict(lambda: defaultdict(float))
        for e in _per_dispatch(path).values():
            c = g[(e["name"], e["grid"])]
            for name, x in e.items():
                if name not in ("name", "grid"):
                    c[name] += x
        return g
    mf, ld = group(a.mfma), group(a.lds)
    fr, wr = read_counters(a.fetch), read_counters(a.write)
    cal = calibration_dispatch(wr)
    fscale = GIB_KIB / float(next(r for r in fr if int(r["Dispatch_Id"]) == cal)["Counter_Value"])
    wscale = GIB_KIB / float(next(r for r in wr if int(r["Dispatch_Id"]) == cal)["Counter_Value"])
    wmap = {int(r["Dispatch_Id"]): float(r["Counter_Value"]) for r in wr}
    hbm = defaultdict(lambda: [0, 0.0])
    for r in fr:
        d = int(r["Dispatch_Id"])
        if d == cal or d not in wmap:
            continue
        k = (short_name(r["Kernel_Name"]), int(r["Grid_Size"]))
        hbm[k][0] += 1
        hbm[k][1] += (float(r["Counter_Value"]) * fscale + wmap[d] * wscale) * 1024.0
    sha = hashlib.sha256(open(os.path.join(ROOT, GEMM_SRC), "rb").read()).hexdigest()[:16]
    lines = [f"# {a.title}", "", "Commands (run from the repository root on one MI355X, ROCm 7.2, "
             "`export TMPDIR=/tmp`):", "", "```"] + a.command + ["```", "",
             f"Kernel source: `{GEMM_SRC}` sha256[:16] = `{sha}`.", "",
             "Columns: kernel and grid (threads); dispatches and average time from the kernel trace; "
             "executed matrix-core work per type (SQ_INSTS_VALU_MFMA_MOPS_<type> x 512 flops, padded tile "
             "rows included) over the dispatch time of the counter run, as "
             "TF/s and as a fraction of that type's dense peak (F64 78.6, F32 157.3, BF16 2500 TF/s); MFMA busy "
             "= SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / 8 x 1024 SIMDs); clock = GRBM_GUI_ACTIVE / 8 over "
             "the dispatch time (dispatches of 0.4 ms or more); LDS conflict = SQ_LDS_BANK_CONFLICT cycles per "
             "SQ_INSTS_LDS instruction; LDS wait = SQ_WAIT_INST_LDS over SQ_WAVE_CYCLES (share of wave time "
             "spent waiting to issue an LDS instruction); HBM = FETCH_SIZE and WRITE_SIZE scaled by a 1 GiB "
             f"device copy (x {fscale:.4f} and x {wscale:.4f}), per dispatch.", "",
             "| kernel | grid | n | avg ms | MFMA type | TF/s | % peak | MFMA busy % | GHz | LDS conflict | "
             "LDS wait % | HBM GB |", "|---|---:|---:|---:|---|---:|---:|---:|---:|---:|---:|---:|"]
    for k in sorted(tr, key=lambda k: -tr[k][1])[:a.top]:
        n, t = tr[k]
        c, l = mf.get(k, {}), ld.get(k, {})
        tf, typ, frac = "", "-", ""
        tm = c.get("t", 0.0)
        for ty in ("F64", "F32", "BF16"):
            m = c.get(f"SQ_INSTS_VALU_MFMA_MOPS_{ty}", 0.0)
            if m > 0 and tm > 0:
                x = m * MOPS_FLOPS[ty] / tm / 1e12
                typ, tf, frac = ty, f"{x:.1f}", f"{100 * x / PEAK_TFS[ty]:.1f}"
        gui = c.get("GRBM_GUI_ACTIVE", 0.0)
        busy = f"{100 * c['SQ_VALU_MFMA_BUSY_CYCLES'] / (gui / 8 * N_SIMD):.1f}" if gui else ""
        clk = f"{gui / 8 / tm / 1e9:.2f}" if gui and tm and tm / max(1, n) > 4e-4 else "-"
        conf = f"{l['SQ_LDS_BANK_CONFLICT'] / l['SQ_INSTS_LDS']:.2f}" if l.get("SQ_INSTS_LDS") else ""
        wait = f"{100 * l['SQ_WAIT_INST_LDS'] / l['SQ_WAVE_CYCLES']:.1f}" if l.get("SQ_WAVE_CYCLES") else ""
        hb = f"{hbm[k][1] / hbm[k][0] / 1e9:.3f}" if hbm.get(k) and hbm[k][0] else ""
        lines.append(f"| `{k[0]}` | {k[1]} | {n} | {t / n * 1e3:.3f} | {typ} | {tf} | {frac} | {busy} | {clk} | "
                     f"{conf} | {wait} | {hb} |")
    os.makedirs(os.path.dirname(os.path.abspath(a.md)), exist_ok=True)
    open(a.md, "w").write("\n".join(lines) + "\n")
    print(f"wrote {a.md}")


if __name__ == "__main__":
    import sys
    if sys.argv[1:2] == ["mfma"]:
        mfma_main(sys.argv[2:])
    elif sys.argv[1:2] == ["kernels"]:
        kernels_main(sys.argv[2:])
    else:
        main()
