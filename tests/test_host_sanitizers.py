"""Host code under sanitizers (CPU only): the oracle, and the library's host
setup (validation, scaling, integer terms, FP64 ILU(0), factor casts, level
sets, SELL-64 layout, blocked sweep schedules), each built with g++ and AddressSanitizer +
UndefinedBehaviorSanitizer, the threaded setup also with ThreadSanitizer.
The drivers (tests/san/) check statuses and, for the setup, that one and four
threads give the same products bit for bit. GPU code is not built here."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ORACLE_SOURCES = ["orc_fx.c", "orc_setup.c", "orc_cycle.c", "orc_ir.c", "orc_gmres64.c"]


def _build_and_run(tmp_path, compiler, flags, sources, name):
    if shutil.which(compiler) is None:
        pytest.skip(f"{compiler} not found")
    exe = str(tmp_path / name)
    cmd = [compiler, *flags, "-o", exe, *sources]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0 and "sanitize" in res.stderr and "cannot find" in res.stderr:
        pytest.skip("sanitizer runtime not installed")
    assert res.returncode == 0, res.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1",
               TSAN_OPTIONS="halt_on_error=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert run.returncode == 0, (run.stdout + run.stderr)[-3000:]
    return run.stdout


def test_oracle_under_asan_ubsan(tmp_path):
    out = _build_and_run(
        tmp_path, "gcc",
        ["-std=c11", "-O1", "-g", "-ffp-contract=off", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
        [os.path.join(HERE, "san", "orc_driver.c")] + [os.path.join(ROOT, "oracle", s) for s in ORACLE_SOURCES]
        + ["-lm"], "orc_san")
    assert "0 failures" in out


HOST_FLAGS = ["-std=c++17", "-O1", "-g", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]
HOST_SOURCES = [os.path.join(HERE, "san", "setup_driver.cpp"),
                os.path.join(ROOT, "paper_2009_07495_amd", "csrc", "igm_setup.cpp"),
                os.path.join(ROOT, "paper_2009_07495_amd", "csrc", "igm_bsched.cpp"), "-lpthread"]


def test_host_setup_under_asan_ubsan(tmp_path):
    out = _build_and_run(tmp_path, "g++", HOST_FLAGS + ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
                         HOST_SOURCES, "setup_asan")
    assert "0 failures" in out


def test_host_setup_under_tsan(tmp_path):
    out = _build_and_run(tmp_path, "g++", HOST_FLAGS + ["-fsanitize=thread"], HOST_SOURCES, "setup_tsan")
    assert "0 failures" in out
