"""The oracle under gcc's AddressSanitizer and UndefinedBehaviorSanitizer:
oracle/sanitize_check.c calls every oracle entry point (right-hand sides,
monitors, Runge-Kutta runs, the sub-cycled hierarchy step in every mode,
regrid, radiative boundaries, prolongation and restriction, the adjoint) on
small ragged inputs; any out-of-bounds access, use after free, leak or
undefined operation aborts it."""
import os
import shutil
import subprocess
from pathlib import Path

import pytest

ORACLE = Path(__file__).resolve().parents[1] / "oracle"
C_SRC = ["orc_core.c", "orc_stencil.c", "orc_mhd.c", "orc_ccz4.c", "orc_amr.c", "orc_adjoint.c",
         "orc_monitor.c", "sanitize_check.c"]
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (cmd, r.stdout[-4000:], r.stderr[-4000:])
    return r


def test_oracle_is_clean_under_asan_and_ubsan(tmp_path):
    if shutil.which("gcc") is None or shutil.which("g++") is None:
        pytest.skip("gcc/g++ not available")
    objs = []
    for src in C_SRC:
        o = tmp_path / (Path(src).stem + ".o")
        _run(["gcc", "-O2", "-g", "-std=c99", "-ffp-contract=off", "-Wall", "-Wextra", "-Wno-unused-parameter",
              *SAN, "-I", str(ORACLE), "-c", str(ORACLE / src), "-o", str(o)])
        objs.append(str(o))
    o = tmp_path / "orc_ccz4_jvp.o"
    _run(["g++", "-O2", "-g", "-std=c++17", "-ffp-contract=off", *SAN, "-I", str(ORACLE), "-c",
          str(ORACLE / "orc_ccz4_jvp.cpp"), "-o", str(o)])
    objs.append(str(o))
    exe = tmp_path / "sanitize_check"
    _run(["g++", *SAN, "-o", str(exe), *objs, "-lm"])
    # verify_asan_link_order=0: the environment may preload other libraries
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = _run([str(exe)], env=env, timeout=600)
    assert r.stdout.strip().endswith("clean (0 failures)"), r.stdout
