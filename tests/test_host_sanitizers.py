"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only).

A second build of libdgw.so instruments the host side only (mesh checks,
reference element, geometry, face matching, renumbering, argument checks of
every entry point); device code is compiled as usual.  The host-ABI tests
then run against it in a child process with the ASan runtime preloaded, and
must pass with no sanitizer report."""

import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1304_5546_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

pytestmark = pytest.mark.slow


def _asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def _build(outdir):
    objs = []
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))
    procs = []
    for src in srcs:
        obj = os.path.join(outdir, os.path.basename(src) + ".o")
        cmd = [HIPCC, "-O1", "-g", "-fno-omit-frame-pointer", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
               "-I", os.path.join(ROOT, "include"), "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
               "-Xarch_host", "-fno-sanitize-recover=undefined"]
        if src.endswith(".cpp"):
            cmd += ["-x", "hip"]
        cmd += ["-c", src, "-o", obj]
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
        objs.append(obj)
    for p in procs:
        out, _ = p.communicate()
        assert p.returncode == 0, out
    lib = os.path.join(outdir, "libdgw_hostsan.so")
    link = [HIPCC, "-shared", "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address",
            "-Xarch_host", "-fsanitize=undefined", "-o", lib, *objs]
    r = subprocess.run(link, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    return lib


def test_host_abi_tests_under_asan_and_ubsan(tmp_path):
    rt = _asan_runtime()
    if rt is None or not os.path.exists(HIPCC):
        pytest.skip("no hipcc or ASan runtime in this image")
    lib = _build(str(tmp_path))
    syms = subprocess.run(["nm", "-D", "--undefined-only", lib], capture_output=True, text=True).stdout
    assert "__asan_report" in syms and "__ubsan_handle" in syms, "host code is not instrumented"
    env = dict(os.environ)
    env.update({"DGW_LIB": lib, "DGW_NO_TORCH": "1", "LD_PRELOAD": rt,
                "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0",
                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"})
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi_host.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    print(out[-3000:])
    assert r.returncode == 0, out[-3000:]
    assert "AddressSanitizer" not in out and "runtime error:" not in out
