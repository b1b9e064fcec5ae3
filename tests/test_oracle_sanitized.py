"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: oracle/sanitize_check.c runs
geometry, viscosity, an RK2 step with each end-of-stage projection, the drags, the nodal
operators and the step and drag adjoints on a sphere, a rotated ellipsoid, an EB slab, a
cylinder and two fluid cavities (one of them on a coarse box, whose wall stencils take the
covered-node fallback), built with -fsanitize=address,undefined and no recovery: any
out-of-bounds access, use after free, leak or undefined arithmetic ends the run with a report
and a non-zero status."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")


def test_oracle_clean_under_asan_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    exe = str(tmp_path / "sanitize_check")
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-Wall", "-Wno-unknown-pragmas", "-ffp-contract=off",
           "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", ORACLE, os.path.join(ORACLE, "eb_oracle.c"),
           os.path.join(ORACLE, "sanitize_check.c"), "-o", exe, "-lm"]
    b = subprocess.run(cmd, capture_output=True, text=True)
    assert b.returncode == 0, b.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    out = r.stdout + r.stderr
    print(r.stdout)
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
    lines = {l.split(":")[0]: l for l in r.stdout.splitlines() if ":" in l}
    assert set(lines) == {"sphere", "ellipsoid", "zslab", "cylinder", "cavity",
                          "cavity_fallback"}, r.stdout
    nfb = int(lines["cavity_fallback"].split("nfallback")[1].split(",")[0])
    assert nfb > 0, lines["cavity_fallback"]
