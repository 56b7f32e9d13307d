"""The CPU-side code under AddressSanitizer and UndefinedBehaviorSanitizer.

Two builds of the same sources: the oracle with gcc's sanitizers, and the
host code of the HIP library with clang's (its device code as usual, and no
GPU is touched).  Each runs the CPU tests that exercise it in a child process
with the sanitizer runtime preloaded; any report (an out-of-bounds access, a
use after free, undefined behaviour, which aborts) fails the test.  Leak
checking is off: the Python interpreter itself holds memory until exit."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

REPORTS = ("ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer")


def run_under(preload, env_extra, tests, timeout):
    env = dict(os.environ)
    env.update(env_extra)
    env["LD_PRELOAD"] = " ".join(preload)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["OMP_NUM_THREADS"] = "4"
    cmd = [sys.executable, "-m", "pytest", *tests, "-x", "-q", "-m", "not gpu", "-p", "no:cacheprovider"]
    p = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    out = p.stdout + p.stderr
    print(out[-3000:])
    assert p.returncode == 0, out[-3000:]
    assert not any(r in out for r in REPORTS), out[-3000:]
    assert " passed" in out


def gcc_runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip(f"gcc runtime {name} not found")
    return path


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    import oracle
    lib = oracle.build(out=str(tmp_path / "libccmg_oracle_san.so"), sanitize=True)
    tests = [os.path.join("tests", f) for f in sorted(os.listdir(os.path.join(ROOT, "tests")))
             if f.startswith("test_oracle_")]
    run_under([gcc_runtime("libasan.so"), gcc_runtime("libubsan.so")], {"CCMG_ORACLE_LIB": lib}, tests, 1500)


def test_host_library_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    from paper_1410_6609_amd import build as hipbuild
    rt = subprocess.run([hipbuild.hipcc(), "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                        text=True).stdout.strip()
    if not os.path.isabs(rt) or not os.path.exists(rt):
        pytest.skip("clang's ASan runtime not found")
    lib = hipbuild.build(out=str(tmp_path / "libccmg_san.so"), sanitize_host=True)
    run_under([rt], {"CCMG_LIB": lib}, [os.path.join("tests", "test_abi_host.py")], 600)
