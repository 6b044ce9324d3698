"""Host code of libppl under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The four HIP sources are compiled with both sanitizers on their host code (the device code
is built as usual and never runs here), linked with the check program tests/native/
host_check.cpp, and run without a GPU: the planner over many shapes, precisions, budgets
and flags, the tune-cache parser on malformed files, the batched and MLP handles, the
argument and state errors of the device entry points, and the DIIS subspace solve. Any
memory error, undefined behaviour or failed check fails the test. The objects are cached
under tests/native/_build and rebuilt when a source or the flags change.
"""
import hashlib
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2603_20912_amd", "csrc")
INC = os.path.join(ROOT, "include")
NATIVE = os.path.join(ROOT, "tests", "native")
BUILD = os.path.join(NATIVE, "_build")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"
# host-side sanitizers only: each one passed to the host compilation alone
HIP_FLAGS = ["--offload-arch=gfx950", "-O1", "-g", "-fPIC", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined",
             "-I", INC, "-I", CSRC]
HOST_SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]

pytestmark = pytest.mark.slow


def _digest(paths, flags):
    h = hashlib.sha256(" ".join(flags).encode())
    for p in sorted(paths):
        h.update(open(p, "rb").read())
    return h.hexdigest()


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd[:3])} ... failed:\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r


def test_host_code_under_sanitizers():
    if not os.path.exists(CLANG) or not os.path.exists(HIPCC):
        pytest.skip("ROCm clang or hipcc not available")
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))
    heads = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")] + [os.path.join(INC, "ppl.h")]
    stamp = os.path.join(BUILD, "objects.sha256")
    digest = _digest(srcs + heads, HIP_FLAGS)
    objs = [os.path.join(BUILD, os.path.basename(s)[:-4] + ".o") for s in srcs]
    if not (os.path.exists(stamp) and open(stamp).read() == digest and all(map(os.path.exists, objs))):
        procs = [subprocess.Popen([HIPCC, *HIP_FLAGS, "-c", s, "-o", o], stdout=subprocess.PIPE,
                                  stderr=subprocess.PIPE, text=True) for s, o in zip(srcs, objs)]
        for p, s in zip(procs, srcs):
            out, err = p.communicate(timeout=900)
            assert p.returncode == 0, f"hipcc failed on {s}:\n{err[-3000:]}"
        open(stamp, "w").write(digest)
    exe = os.path.join(BUILD, "host_check")
    drv = os.path.join(BUILD, "host_check.o")
    _run([CLANG, "-std=c++17", "-g", *HOST_SAN, "-fno-omit-frame-pointer", "-I", INC, "-I", CSRC, "-c",
          os.path.join(NATIVE, "host_check.cpp"), "-o", drv])
    _run([CLANG, *HOST_SAN, drv, *objs, "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    env = dict(os.environ)
    # LeakSanitizer too: every handle the program creates is destroyed
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["HIP_VISIBLE_DEVICES"] = ""
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
    assert "host checks: 0 of" in r.stdout, out[-4000:]
