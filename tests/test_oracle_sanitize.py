"""The CPU oracle under AddressSanitizer, UndefinedBehaviorSanitizer and the leak checker: a C driver
(tests/oracle_sanitize_main.c) runs every entry point on small problems that reach each code path (1D,
2D, 3D, every boundary kind, Navier-Stokes with the Prandtl fix, the fallbacks, the reading modes, a
three-stage tableau, stage fluxes, unit functions, error returns). Any sanitizer report aborts the run.
The same driver built without sanitizers at the oracle's own optimisation prints the same numbers, so the
sanitized run computed what the oracle computes."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = [os.path.join(ROOT, "oracle", "hgks_oracle.c"), os.path.join(HERE, "oracle_sanitize_main.c")]
COMMON = ["-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-D_GNU_SOURCE",
          "-I", os.path.join(ROOT, "oracle")]


def _build(tmp, name, flags):
    out = os.path.join(tmp, name)
    subprocess.run(["gcc", *COMMON, *flags, *SRC, "-o", out, "-lm"], check=True, capture_output=True,
                   text=True)
    return out


def _run(exe):
    env = dict(os.environ, OMP_NUM_THREADS="3",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    return subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_clean_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    san = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    try:
        exe = _build(str(tmp_path), "drv_san", san)
    except subprocess.CalledProcessError as e:
        if "asan" in e.stderr or "ubsan" in e.stderr:
            pytest.skip("the sanitizer runtimes are not installed: " + e.stderr[-200:])
        raise
    r = _run(exe)
    assert r.returncode == 0 and "sanitize-driver ok" in r.stdout, r.stdout[-2000:] + r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-4000:]
    plain = _run(_build(str(tmp_path), "drv", ["-O2"]))
    assert plain.returncode == 0
    assert plain.stdout == r.stdout
