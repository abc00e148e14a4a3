"""The library's host code under AddressSanitizer (CPU only).

Every source is rebuilt with the sanitizer on the host side only (the GPU code
is compiled as usual and never runs: no device is needed), linked with the C
driver in tests/host_asan/, and run with leak checking (leaks inside the HIP
runtime itself suppressed).  The driver exercises the host logic: index and
size helpers, quantiles, batch work lists, configuration resolution, tuning
candidates and cache parsing (valid, malformed and over-long lines), argument
rejection, stream admission, a stream whose device allocation fails, and the
streaming fold schedule (counted, listed in full and truncated).
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1702_00844_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"
CLANGXX = "/opt/rocm/llvm/bin/clang++"


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm compilers not installed")
def test_host_code_under_address_sanitizer(tmp_path):
    srcs = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    procs, objs = [], []
    for f in srcs:
        obj = str(tmp_path / (f + ".o"))
        objs.append(obj)
        cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer",
               "-Wno-unused-function", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
               "-c", os.path.join(CSRC, f), "-o", obj]
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
    for f, p in zip(srcs, procs):
        out, _ = p.communicate(timeout=600)
        assert p.returncode == 0, f + ":\n" + out
    drv = str(tmp_path / "driver.o")
    r = subprocess.run([CLANG, "-g", "-O1", "-fsanitize=address", "-fno-omit-frame-pointer",
                        "-I", os.path.join(ROOT, "include"), "-c", os.path.join(ROOT, "tests", "host_asan", "driver.c"),
                        "-o", drv], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    exe = str(tmp_path / "driver")
    r = subprocess.run([CLANGXX, "-fsanitize=address", "-o", exe, drv, *objs, "-L/opt/rocm/lib", "-lamdhip64",
                        "-Wl,-rpath,/opt/rocm/lib"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    supp = tmp_path / "lsan.supp"
    supp.write_text("leak:libamdhip64\nleak:libhsa-runtime64\nleak:libamd_comgr\nleak:librocprofiler\n")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", LSAN_OPTIONS="suppressions=%s" % supp)
    r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, timeout=300, env=env)
    assert "AddressSanitizer" not in r.stderr and "LeakSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), (r.returncode, r.stdout, r.stderr[-4000:])
