"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only, no GPU).

- The oracle (plain C) is rebuilt with gcc's -fsanitize=address,undefined
  in a temporary copy of the test tree, and the oracle's CPU tests run there
  with gcc's sanitizer runtimes preloaded.  A planted out-of-bounds write (an
  oracle call given a ranges array too short for the tile ids it is handed)
  must be reported, which shows the instrumentation is live.
- The host side of libxg's C ABI (api.cpp: argument validation, workspace
  layout, launch planning) is rebuilt with the same sanitizers on the host
  pass only (device code is not instrumented) and linked with the other
  objects of the regular build; the C ABI tests run against it with clang's
  ASan runtime preloaded.  They make no HIP call that reaches a device.

Any sanitizer report ends the child process with a nonzero status.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ENV_SAN = {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _gcc_runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def _copy_tree(dst, with_package=False):
    for d in ("oracle", "scenes", "include"):
        shutil.copytree(os.path.join(ROOT, d), os.path.join(dst, d),
                        ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    os.makedirs(os.path.join(dst, "tests"))
    for f in os.listdir(os.path.join(ROOT, "tests")):
        if f.endswith(".py") and (f.startswith("test_oracle") or f in ("conftest.py", "test_abi.py")):
            shutil.copy(os.path.join(ROOT, "tests", f), os.path.join(dst, "tests", f))
    shutil.copytree(os.path.join(ROOT, "tests", "golden"), os.path.join(dst, "tests", "golden"))
    shutil.copy(os.path.join(ROOT, "pytest.ini"), dst)
    if with_package:
        shutil.copytree(os.path.join(ROOT, "paper_2403_04116_amd"), os.path.join(dst, "paper_2403_04116_amd"),
                        ignore=shutil.ignore_patterns("*.so", "_build", "__pycache__"))


def _run(cmd, cwd, preload, timeout=900):
    env = dict(os.environ, **ENV_SAN, LD_PRELOAD=preload)
    return subprocess.run(cmd, cwd=cwd, env=env, capture_output=True, text=True, timeout=timeout)


def test_oracle_under_asan_ubsan(tmp_path):
    asan, ubsan = _gcc_runtime("libasan.so"), _gcc_runtime("libubsan.so")
    if not (asan and ubsan):
        pytest.skip("gcc sanitizer runtimes not installed")
    d = str(tmp_path / "o")
    _copy_tree(d)
    lib = os.path.join(d, "oracle", "liboracle.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-Wall", "-ffp-contract=off", "-fno-fast-math",
                           "-fopenmp", "-fPIC", "-shared", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-o", lib,
                           os.path.join(d, "oracle", "oracle.c"), "-lm"])
    preload = f"{asan} {ubsan}"
    tests = sorted(f"tests/{f}" for f in os.listdir(os.path.join(d, "tests")) if f.startswith("test_oracle"))
    r = _run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", *tests], d, preload)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "passed" in r.stdout
    # positive control: orc_ranges writes ranges[2 g] for tile g = 5 into a
    # 2-word array
    probe = ("import ctypes, numpy as np, oracle as O; L = O.lib(); "
             "k = np.array([5 << 32], np.uint64); r = np.zeros(2, np.uint32); "
             "L.orc_ranges(1, k.ctypes.data_as(ctypes.c_void_p), 1, r.ctypes.data_as(ctypes.c_void_p))")
    r = _run([sys.executable, "-c", probe], d, preload, timeout=300)
    assert r.returncode != 0 and "AddressSanitizer" in r.stderr, r.stderr[-2000:]


def test_abi_host_code_under_asan_ubsan(tmp_path):
    objdir = os.path.join(ROOT, "paper_2403_04116_amd", "_build")
    if not os.path.isdir(objdir) or not os.path.exists(os.path.join(objdir, "render.o")):
        pytest.skip("libxg objects not built (run __graft_entry__.build())")
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not installed")
    rt = subprocess.run([HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                        text=True).stdout.strip()
    if not (os.path.isabs(rt) and os.path.exists(rt)):
        cands = [os.path.join(dp, f) for dp, _, fs in os.walk("/opt/rocm/llvm/lib/clang") for f in fs
                 if f == "libclang_rt.asan-x86_64.so"]
        if not cands:
            pytest.skip("clang ASan runtime not found")
        rt = cands[0]
    d = str(tmp_path / "x")
    _copy_tree(d, with_package=True)
    pkg = os.path.join(d, "paper_2403_04116_amd")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer"]
    api_o = os.path.join(str(tmp_path), "api.o")
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-fPIC", "-std=c++17", "-x", "hip",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *san,
                           f"-I{os.path.join(d, 'include')}", f"-I{os.path.join(pkg, 'csrc')}", "-c",
                           os.path.join(pkg, "csrc", "api.cpp"), "-o", api_o])
    objs = [os.path.join(objdir, f) for f in sorted(os.listdir(objdir)) if f.endswith(".o") and f != "api.o"]
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *san, "-shared-libasan",
                           "-o", os.path.join(pkg, "libxg.so"), api_o, *objs])
    r = _run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "tests/test_abi.py"], d, rt)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "passed" in r.stdout
