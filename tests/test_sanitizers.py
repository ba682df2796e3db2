"""The oracle and the library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only): each suite runs in a child process that preloads
the sanitizer runtime and loads the sanitized build; any report fails the run."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(env_extra, tests):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"      # the interpreter keeps objects
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu", *tests], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=1500)
    print(r.stdout[-2000:], r.stderr[-2000:])
    assert r.returncode == 0
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr


@pytest.mark.slow
def test_oracle_under_asan_ubsan():
    from oracle import oracle as O
    O.build(force=True, sanitize=True)
    gcc = lambda name: subprocess.check_output(["gcc", f"-print-file-name={name}"], text=True).strip()
    run({"LD_PRELOAD": f"{gcc('libasan.so')}:{gcc('libubsan.so')}", "BBX_ORACLE_SANITIZE": "1"},
        ["tests/test_oracle_stencil.py", "tests/test_oracle_tips.py", "tests/test_oracle_rk4.py",
         "tests/test_oracle_ecg.py", "tests/test_oracle_kinetics.py", "tests/test_oracle_mlp.py"])


@pytest.mark.slow
def test_host_code_under_asan_ubsan():
    from paper_1605_06015_amd import build as Bd
    lib = Bd.build(sanitize=True)
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt:
        pytest.skip("clang's ASan runtime is not installed")
    run({"LD_PRELOAD": rt[-1], "BBX_LIB": lib}, ["tests/test_abi_host.py"])
