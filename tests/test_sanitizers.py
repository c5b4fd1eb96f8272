"""CPU builds under AddressSanitizer and UndefinedBehaviorSanitizer: the
oracle (gcc) driven through every entry point on small inputs, and the host
side of libgj (argument checks, batch plans, workspace sizes) driven through
its C ABI with no GPU call.  A sanitizer report aborts the driver, which
fails the test."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:verify_asan_link_order=0",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def test_oracle_asan_ubsan(tmp_path):
    exe = tmp_path / "oracle_driver"
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", "-o", str(exe),
                    os.path.join(HERE, "oracle_driver.c"), os.path.join(ROOT, "oracle", "gj_oracle.c"),
                    "-lm"], check=True)
    env = dict(os.environ, OMP_NUM_THREADS="4", **SAN_ENV)
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "oracle driver: done" in r.stdout


def _asan_runtime():
    out = subprocess.run(["/opt/rocm/bin/hipcc", "--print-file-name=libclang_rt.asan-x86_64.so"],
                         capture_output=True, text=True).stdout.strip()
    if out and os.path.isabs(out) and os.path.exists(out):
        return out
    base = "/opt/rocm/lib/llvm/lib/clang"
    if os.path.isdir(base):
        for v in sorted(os.listdir(base)):
            p = os.path.join(base, v, "lib", "linux", "libclang_rt.asan-x86_64.so")
            if os.path.exists(p):
                return p
    return None


def test_host_plans_asan_ubsan(tmp_path):
    """api.hip's host code instrumented (device code as usual), linked with
    the regular objects of the other sources."""
    from paper_1401_7962_amd import build as B
    rt = _asan_runtime()
    if rt is None or not os.path.exists(B.HIPCC):
        pytest.skip("no hipcc / clang ASan runtime in this image")
    objs = [os.path.join(B.BUILD_DIR, os.path.splitext(x)[0] + ".o") for x in B.SOURCES
            if x != "api.hip"]
    if not all(os.path.exists(o) for o in objs):
        B.build()
    api_o = tmp_path / "api_san.o"
    flags = [f for f in B.FLAGS if f != "-O3"] + ["-O1", "-g", "-fno-omit-frame-pointer"]
    subprocess.run([B.HIPCC, *flags, "-Xarch_host", "-fsanitize=address",
                    "-Xarch_host", "-fsanitize=undefined",
                    "-Xarch_host", "-fno-sanitize-recover=all",
                    "-c", os.path.join(B.CSRC, "api.hip"), "-o", str(api_o)], check=True)
    lib = tmp_path / "libgj_san.so"
    subprocess.run([B.HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC",
                    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                    "-o", str(lib), str(api_o), *objs], check=True)
    shutil.copy(os.path.join(B.HERE, "gj_tune.txt"), tmp_path / "gj_tune.txt")
    env = dict(os.environ, LD_PRELOAD=rt, **SAN_ENV)
    r = subprocess.run([sys.executable, os.path.join(HERE, "host_abi_driver.py"), str(lib)],
                       capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "host driver: done" in r.stdout
