"""The FP64 oracle and the C ABI's host code under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only).

* The oracle with its own driver (oracle/sanitizer_driver.c: every entry
  point on small ERP, pinhole and row-crop scenes with seam straddlers, ties
  and near-threshold decisions), built with gcc's sanitizers.
* The library's host code: capi.hip recompiled with the sanitizers on its
  host pass only (the device code is unchanged), linked with the other
  objects, and the host-side contract tests (tests/test_capi_host.py) run
  against it in a child process that preloads the sanitizer runtime.
"""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_ENV = dict(ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_san")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-ffp-contract=off", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-o", exe,
           os.path.join(ROOT, "oracle", "sanitizer_driver.c"), "-lm"]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "sanitized oracle run ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr


def _asan_runtime():
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return found[-1] if found else None


@pytest.mark.slow
def test_capi_host_code_under_asan_and_ubsan(tmp_path):
    from paper_2404_03202_amd import build as b
    rt = _asan_runtime()
    if rt is None or shutil.which(b.hipcc()) is None and not os.path.exists(b.hipcc()):
        pytest.skip("no hipcc or clang sanitizer runtime")
    objdir = os.path.join(b.HERE, "_build")
    others = [os.path.join(objdir, s.replace(".hip", ".o")) for s in b.SOURCES if s != "capi.hip"]
    if not all(os.path.exists(o) for o in others):
        pytest.skip("library objects not built: run `python -m paper_2404_03202_amd.build`")
    capi = str(tmp_path / "capi.o")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host",
           "-fno-omit-frame-pointer", "-g"]
    subprocess.run([b.hipcc(), *b.HIPCC_FLAGS, *san, "-I", b.INCLUDE, "-c", os.path.join(b.CSRC, "capi.hip"), "-o",
                    capi], check=True, capture_output=True)
    lib = str(tmp_path / "libomnigs_san.so")
    subprocess.run([b.hipcc(), f"--offload-arch={b.ARCH}", "-shared", "-fPIC", "-o", lib, capi, *others], check=True,
                   capture_output=True)
    script = (f"import sys; sys.path.insert(0, {ROOT!r}); "
              f"from paper_2404_03202_amd import omnigs as B; B.load_library({lib!r}); import pytest; "
              f"sys.exit(pytest.main(['-q', '-x', '-p', 'no:cacheprovider', "
              f"{os.path.join(ROOT, 'tests', 'test_capi_host.py')!r}]))")
    env = dict(os.environ, LD_PRELOAD=rt, **SAN_ENV)
    r = subprocess.run([sys.executable, "-c", script], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "passed" in r.stdout and "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
