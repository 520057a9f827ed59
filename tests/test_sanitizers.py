"""The CPU tests under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle (plain C) and the host code of librflbm (the C interface, batch
and run-time logic; device code is built as usual) are rebuilt with
-fsanitize=address,undefined, and the C-interface, table, generator and
collision pins run against those builds in a child process with clang's ASan
runtime preloaded.  Any sanitizer report fails the run (UBSan halts on the
first error).  The whole CPU suite runs the same way with
RFLBM_LIBRARY / RFLBM_ORACLE_LIBRARY set to the two builds."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SUBSET = ["tests/test_abi.py", "tests/test_oracle_tables.py", "tests/test_oracle_collide.py",
          "tests/test_philox.py", "tests/test_oracle_recursive.py"]


def asan_runtime():
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return found[-1] if found else None


@pytest.mark.slow
def test_cpu_suite_clean_under_address_and_undefined_sanitizers(tmp_path):
    rt = asan_runtime()
    if rt is None:
        pytest.skip("clang ASan runtime not found")
    sys.path.insert(0, ROOT)
    import oracle
    from paper_2507_08820_amd import build as gpu_build

    ora_lib = oracle.build(sanitize=True, out=str(tmp_path / "liboracle_asan.so"))
    lib = gpu_build.build(out=str(tmp_path / "librflbm_asan.so"), build_dir=str(tmp_path / "build"),
                          sanitize_host=True)
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               RFLBM_LIBRARY=lib, RFLBM_ORACLE_LIBRARY=ora_lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu and not slow"]
                       + SUBSET, cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-3000:]
    assert r.returncode == 0, out[-3000:]
    assert " passed" in out
