"""AddressSanitizer + UndefinedBehaviorSanitizer runs of the host code, on the CPU:

* the oracle (plain C, gcc) driven through every exported function on small inputs
  (tests/sanitize/oracle_driver.c);
* the library's host side (argument checks, planning, reports, the error paths of
  every entry point without a GPU), built with hipcc with the sanitizers on the host
  code only, linked with the built kernels (tests/sanitize/runtime_driver.cpp).
"""
import os
import shutil
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
SAN = ROOT / "tests" / "sanitize"
CSRC = ROOT / "paper_1003_2022_amd" / "csrc"
HOST_SOURCES = ["svf_runtime.cpp", "svf_batch.cpp", "svf_server.cpp", "svf_st.cpp"]
KERNEL_OBJS = ["svf_kernels.hip.o", "svf_fd.hip.o", "svf_st.hip.o", "svf_noalloc.hip.o", "svf_single.hip.o"]


def run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    return r.returncode, r.stdout + r.stderr


def test_oracle_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_driver"
    rc, out = run(["gcc", "-O1", "-g", "-std=gnu11", "-ffp-contract=off", "-fopenmp", "-fsanitize=address,undefined",
                   "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", str(ROOT / "oracle" / "svf_oracle.c"),
                   str(SAN / "oracle_driver.c"), "-o", str(exe), "-lm"])
    if rc != 0 and "sanitize" in out and "cannot find" in out:
        pytest.skip("gcc sanitizer runtimes not installed")
    assert rc == 0, out
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", OMP_NUM_THREADS="2")
    rc, out = run([str(exe)], env=env)
    print(out)
    assert rc == 0, out
    assert "all checks passed" in out


def test_runtime_host_under_sanitizers(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc"
    objs_dir = ROOT / "paper_1003_2022_amd" / "_build"
    if not Path(hipcc).exists():
        pytest.skip("hipcc not available")
    if not all((objs_dir / o).exists() for o in KERNEL_OBJS):
        from paper_1003_2022_amd import build

        build.build()
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++20", "-fPIC", "-Wno-unused-command-line-argument",
             "-Wno-unused-result", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-I", str(ROOT / "include"), "-I", str(CSRC)]
    objs = []
    procs = []
    for src in [SAN / "runtime_driver.cpp"] + [CSRC / s for s in HOST_SOURCES]:
        o = tmp_path / (src.name + ".o")
        objs.append(o)
        procs.append(subprocess.Popen([hipcc, *flags, "-c", str(src), "-o", str(o)], stdout=subprocess.PIPE,
                                      stderr=subprocess.STDOUT, text=True))
    for p in procs:
        out, _ = p.communicate(timeout=600)
        assert p.returncode == 0, out
    exe = tmp_path / "runtime_driver"
    rc, out = run([hipcc, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
                   "-fsanitize=undefined", *map(str, objs), *[str(objs_dir / o) for o in KERNEL_OBJS], "-o", str(exe)])
    assert rc == 0, out
    # the HIP runtime keeps allocations until exit: leak detection off; no GPU is used
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               HIP_VISIBLE_DEVICES="-1")
    rc, out = run([str(exe)], env=env, timeout=300)
    print(out)
    assert rc == 0, out
    assert "all checks passed" in out
